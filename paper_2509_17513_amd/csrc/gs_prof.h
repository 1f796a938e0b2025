// Optional per-kernel timing with HIP events recorded on the launch stream.
#pragma once

#include <hip/hip_runtime.h>

namespace gs {

enum KernelId {
  K_COMPOSE_FWD = 0,
  K_PROJECT_FWD,
  K_RADIX_HIST,
  K_RADIX_SCAN,
  K_RADIX_SCATTER,
  K_BIN_COUNT,
  K_BIN_CHUNK_SCAN,
  K_TILE_RANGES,
  K_BIN_EMIT,
  K_RASTER_FWD,
  K_ZERO,
  K_RASTER_BWD,
  K_PROJECT_BWD,
  K_COMPOSE_BWD,
  K_RATE_CTX,
  K_RATE_MLP,
  K_RATE_HIST_MINMAX,
  K_RATE_HIST_COUNT,
  K_RATE_HIST_BITS,
  K_ADAM,
  K_BIN_GATHER,
  K_ROW_COUNT,
  K_ROW_EMIT,
  K_SSIM_FWD,
  K_SSIM_BWD,
  K_PSI,
  K_MAPS_RANGE,
  K_MAPS_KEYS,
  K_MAPS_WRITE,
  K_MAPS_DECODE,
  K_ENT_STATS,
  K_ENT_HIST,
  K_ENT_CDF,
  K_ENT_EVAL,
  K_MOTION_FWD,
  K_MOTION_BWD,
  K_MOTION_WGRAD,
  K_MOTION_TABLE,
  K_COUNT
};

// Returns a slot handle (or -1 when profiling is off); launches between
// prof_begin and prof_end on `st` are attributed to `id`.
int prof_begin(int id, hipStream_t st);
void prof_end(int slot, hipStream_t st);

struct ProfScope {
  int slot;
  hipStream_t st;
  ProfScope(int id, hipStream_t s) : slot(prof_begin(id, s)), st(s) {}
  ~ProfScope() { prof_end(slot, st); }
};

}  // namespace gs
