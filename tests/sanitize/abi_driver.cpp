// Calls the host-side argument checks of libgs4d.so with invalid and edge-case arguments (none
// reaches a kernel launch); built with AddressSanitizer and UndefinedBehaviorSanitizer on the
// host code by tests/test_sanitizers.py. Exits 0 when every call returns the expected code.
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "gs4d.h"

static int bad = 0;
static void expect(int got, int want, const char* what) {
  if (got != want) {
    std::printf("%s: got %d, want %d\n", what, got, want);
    bad = 1;
  }
}

int main() {
  gs_settings s;
  std::memset(&s, 0, sizeof(s));
  s.width = 64; s.height = 48; s.sh_degree = 0; s.n_levels = 1; s.level_counts[0] = 100;
  s.level_weights[0] = 1.f; s.near_plane = 0.2f; s.dilation = 0.3f; s.alpha_min = 1.f / 255.f;
  s.alpha_max = 0.99f; s.t_stop = 1e-4f;
  size_t bytes = 0;
  expect(gs_workspace_size(&s, 100, 1, 2, 1000, &bytes), GS_OK, "workspace size");
  expect(gs_workspace_size(nullptr, 100, 1, 2, 1000, &bytes), GS_ERR_INVALID_ARG, "NULL settings");
  expect(gs_workspace_size(&s, -1, 1, 2, 1000, &bytes), GS_ERR_INVALID_ARG, "negative n");
  expect(gs_workspace_size(&s, 100, 1, 2, -5, &bytes), GS_ERR_INVALID_ARG, "negative capacity");
  gs_settings t = s;
  t.alpha_max = 1.f;
  expect(gs_workspace_size(&t, 100, 1, 2, 1000, &bytes), GS_ERR_INVALID_ARG, "alpha_max = 1");
  t = s;
  t.n_levels = 9;
  expect(gs_workspace_size(&t, 100, 1, 2, 1000, &bytes), GS_ERR_INVALID_ARG, "nine levels");
  t = s;
  t.width = 4097 * 16;
  expect(gs_workspace_size(&t, 100, 1, 1, 1000, &bytes), GS_ERR_UNSUPPORTED, "too wide");
  char dummy[64];
  expect(gs_render_forward(&s, 100, (const float*)dummy, 1, nullptr, 1, (const gs_camera*)dummy, nullptr, dummy,
                           1 << 20, nullptr), GS_ERR_INVALID_ARG, "NULL image");
  expect(gs_render_forward(&s, 100, (const float*)dummy, 1, nullptr, 1, (const gs_camera*)dummy, (float*)dummy,
                           dummy, 16, nullptr), GS_ERR_WORKSPACE, "small workspace");
  expect(gs_rate_histogram_workspace_size(0, &bytes), GS_ERR_INVALID_ARG, "histogram without attributes");
  std::printf("abi driver: %s; last error \"%s\"\n", bad ? "unexpected code" : "ok", gs_last_error());
  return bad;
}
