// Runs every entry point of the FP64 oracle once on small seeded scenes, including degenerate
// Gaussians (NaN parameters, a zero quaternion, one on the near plane, one behind the camera),
// frame residuals and a pixel sample; built with AddressSanitizer and UndefinedBehaviorSanitizer
// by tests/test_sanitizers.py. Exits 0 when every call returns 0.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

extern "C" {
typedef struct {
  int32_t width, height, sh_degree, n_levels;
  int32_t level_counts[8];
  int32_t res_channels;
  int32_t pad_;
  double near_plane, dilation, alpha_min, alpha_max, t_stop;
  double bg[3];
  double band_safety;
} oc_settings;
int oc_project(const oc_settings*, int, const float*, int, const float*, int, const float*, double*);
int oc_render(const oc_settings*, int, const float*, int, const float*, int, const float*, int, int64_t,
              const int64_t*, double*, double*, int32_t*, uint64_t*, int32_t*, double*);
int oc_backward(const oc_settings*, int, const float*, int, const float*, int, const float*, int, const double*,
                double*, double*, double*);
int oc_backward_abs(const oc_settings*, int, const float*, int, const float*, int, const double*, double*, double*);
int oc_fd(const oc_settings*, int, const float*, int, const float*, const double*, int64_t, const int32_t*,
          const int32_t*, double, double*, int32_t*, int64_t*);
int oc_set_threads(int);
}

int main() {
  const int n = 40, W = 24, H = 20, deg = 1, C = 11 + 3 * 4, V = 2, F = 2, Rc = 8, L = 2;
  std::mt19937 rng(7);
  std::uniform_real_distribution<float> uni(-1.f, 1.f);
  std::normal_distribution<float> nrm(0.f, 1.f);
  std::vector<float> P((size_t)C * n);
  for (int i = 0; i < n; ++i) {
    P[0 * n + i] = uni(rng) * 0.6f;
    P[1 * n + i] = uni(rng) * 0.4f;
    P[2 * n + i] = 3.f + uni(rng);
    for (int c = 3; c < 6; ++c) P[c * n + i] = -2.0f + 0.3f * nrm(rng);
    for (int c = 6; c < 10; ++c) P[c * n + i] = nrm(rng);
    P[10 * n + i] = nrm(rng);
    for (int c = 11; c < C; ++c) P[c * n + i] = 0.3f * nrm(rng);
  }
  P[0 * n + 1] = NAN;        // non-finite mean
  P[11 * n + 2] = NAN;       // non-finite colour
  for (int c = 6; c < 10; ++c) P[c * n + 3] = 0.f;  // zero quaternion
  P[2 * n + 4] = 0.2f;       // on the near plane
  P[2 * n + 5] = -1.f;       // behind the camera
  std::vector<float> res((size_t)F * Rc * n);
  for (auto& x : res) x = 0.01f * nrm(rng);
  for (int f = 0; f < F; ++f)
    for (int i = 0; i < n; ++i) res[((size_t)f * Rc + 3) * n + i] = 1.f;  // delta quaternion near identity
  std::vector<float> cams((size_t)F * V * 16, 0.f);
  for (int b = 0; b < F * V; ++b) {
    float* k = &cams[16 * b];
    k[0] = k[5] = k[10] = 1.f;
    k[3] = 0.05f * (b % V);
    k[12] = k[13] = (float)W;
    k[14] = W / 2.f;
    k[15] = H / 2.f;
  }
  oc_settings s{};
  s.width = W; s.height = H; s.sh_degree = deg; s.n_levels = L;
  s.level_counts[0] = n / 2; s.level_counts[1] = n;
  s.res_channels = Rc;
  s.near_plane = 0.2f; s.dilation = 0.3f; s.alpha_min = 1.0 / 255.0; s.alpha_max = 0.99f; s.t_stop = 1e-4f;
  s.band_safety = 2.0;
  int bad = 0;
  for (int threads : {1, 3}) {
    oc_set_threads(threads);
    const int B = F * V;
    std::vector<double> proj((size_t)B * n * 16);
    bad |= oc_project(&s, n, P.data(), F, res.data(), V, cams.data(), proj.data()) != 0;
    const int64_t npix = (int64_t)W * H;
    std::vector<double> img((size_t)B * L * 3 * npix), T((size_t)B * L * npix), var((size_t)B * L * npix * 16 * 3);
    std::vector<int32_t> nc((size_t)B * L * npix), nvar((size_t)B * L * npix);
    std::vector<uint64_t> sig((size_t)B * L * npix);
    for (int mode = 0; mode < 2; ++mode)
      bad |= oc_render(&s, n, P.data(), F, res.data(), V, cams.data(), mode, 0, nullptr, img.data(), T.data(),
                       nc.data(), sig.data(), nvar.data(), var.data()) != 0;
    std::vector<int64_t> sample = {0, 5, 77, npix - 1};
    std::vector<double> img_s((size_t)B * L * 3 * 4);
    bad |= oc_render(&s, n, P.data(), F, res.data(), V, cams.data(), 0, 4, sample.data(), img_s.data(), nullptr,
                     nullptr, nullptr, nullptr, nullptr) != 0;
    std::vector<double> dimg(img.size());
    for (auto& x : dimg) x = nrm(rng);
    std::vector<double> dp((size_t)C * n), dr((size_t)F * Rc * n), g2((size_t)B * n * 9);
    bad |= oc_backward(&s, n, P.data(), F, res.data(), V, cams.data(), 0, dimg.data(), dp.data(), dr.data(),
                       g2.data()) != 0;
    oc_settings s1 = s;
    s1.res_channels = 0;
    std::vector<double> dimg1((size_t)V * L * 3 * npix), da((size_t)C * n);
    for (auto& x : dimg1) x = nrm(rng);
    bad |= oc_backward_abs(&s1, n, P.data(), V, cams.data(), 1, dimg1.data(), dp.data(), da.data()) != 0;
    std::vector<int32_t> gi, ci;
    for (int i = 0; i < n; i += 3)
      for (int c = 0; c < C; c += 5) { gi.push_back(i); ci.push_back(c); }
    std::vector<double> fd(gi.size());
    std::vector<int32_t> st(gi.size());
    std::vector<int64_t> sk(gi.size());
    bad |= oc_fd(&s1, n, P.data(), V, cams.data(), dimg1.data(), (int64_t)gi.size(), gi.data(), ci.data(), 1e-5,
                 fd.data(), st.data(), sk.data()) != 0;
  }
  std::printf("oracle driver: %s\n", bad ? "a call failed" : "ok");
  return bad;
}
