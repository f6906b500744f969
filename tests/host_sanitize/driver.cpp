// Host-side argument checks of every C ABI entry point, run without a GPU
// under AddressSanitizer and UndefinedBehaviorSanitizer.  The library's host
// runtime (masw_runtime.hip, masw_server.hip) is linked with stub kernel
// launchers: every call below is rejected by its checks before any launch,
// and a launcher that is reached anyway fails the run.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "masw.h"
#include "masw_host.hpp"

namespace masw {
static hipError_t reached(const char* what) {
  std::fprintf(stderr, "stub launcher reached: %s\n", what);
  std::abort();
}
int sweep_blocks_per_cu(int, int) { return 1; }
int tick_blocks_per_cu(int, bool) { return 1; }
hipError_t launch_sweep(int, int, int, hipStream_t, const SweepArgs&) { return reached("sweep"); }
hipError_t launch_fused(int, int, hipStream_t, const SweepArgs&) { return reached("fused sweep"); }
hipError_t launch_inertia(const SweepArgs&, int, hipStream_t, int*) { return reached("inertia"); }
hipError_t launch_prep(const PrepArgs&, const CoopInitArgs&, int, int, hipStream_t) { return reached("prep"); }
hipError_t launch_sign_map(bool, const SignMapArgs&, hipStream_t) { return reached("sign map"); }
hipError_t launch_admit(const AdmitList*, int, int, int32_t*, hipStream_t) { return reached("admit"); }
hipError_t launch_tick(int, int, hipStream_t, const TickArgs&) { return reached("tick"); }
hipError_t launch_misfit(int, const int32_t*, const double*, const double*, double*, hipStream_t) {
  return reached("misfit");
}
hipError_t launch_classify(const ClassifyArgs&, hipStream_t) { return reached("classify"); }
hipError_t launch_serve_noise(const ServeNoiseList&, const int32_t*, int32_t*, double, hipStream_t) {
  return reached("serve noise");
}
hipError_t setup_scratch(int) { return reached("scratch set-up"); }
void* scratch_of(int) {
  reached("scratch address");
  return nullptr;
}
hipError_t launch_noise_check(const ModelDesc*, const LayerRec64*, const double*, const double*, const int32_t*,
                              const int32_t*, int32_t*, int64_t, double, hipStream_t) {
  return reached("noise");
}
}  // namespace masw

static int checks = 0, failures = 0;

static void expect(int rc, int want, const char* what) {
  ++checks;
  if (rc != want) {
    ++failures;
    std::fprintf(stderr, "FAIL %s: rc %d, want %d (%s)\n", what, rc, want, masw_last_error());
  }
}

int main() {
  // a valid two-layer model and grid
  const double h[2] = {2.0, 4.0};
  const double beta[3] = {150.0, 250.0, 400.0};
  double alpha[3], rho[3] = {1850.0, 1900.0, 2000.0};
  for (int j = 0; j < 3; ++j) alpha[j] = std::sqrt(3.0) * beta[j];
  std::vector<double> c(801), lam(30);
  for (int i = 0; i < 801; ++i) c[i] = 50.0 + 0.5 * i;
  for (int i = 0; i < 30; ++i) lam[i] = 1.0 + i;
  std::vector<double> ct(30), cref(30);
  std::vector<int32_t> idx(30), st(30);
  masw_model m{2, h, alpha, beta, rho};

  // curve: each bad argument, then a null context with good arguments
  const int E = MASW_EINVAL;
  expect(masw_dispersion_curve(nullptr, c.data(), 1, lam.data(), 30, &m, MASW_PREC_FP64, 0, nullptr, ct.data(),
                               idx.data(), st.data(), cref.data()), E, "n_c < 2");
  std::vector<double> bad_c = c;
  bad_c[400] = bad_c[399];
  expect(masw_dispersion_curve(nullptr, bad_c.data(), 801, lam.data(), 30, &m, MASW_PREC_FP64, 0, nullptr,
                               ct.data(), idx.data(), st.data(), cref.data()), E, "grid not increasing");
  bad_c[400] = NAN;
  expect(masw_dispersion_curve(nullptr, bad_c.data(), 801, lam.data(), 30, &m, MASW_PREC_FP64, 0, nullptr,
                               ct.data(), idx.data(), st.data(), cref.data()), E, "NaN in grid");
  std::vector<double> bad_l = lam;
  bad_l[7] = -1.0;
  expect(masw_dispersion_curve(nullptr, c.data(), 801, bad_l.data(), 30, &m, MASW_PREC_FP64, 0, nullptr, ct.data(),
                               idx.data(), st.data(), cref.data()), E, "negative wavelength");
  double bad_alpha[3] = {alpha[0], 200.0, alpha[2]};
  masw_model bm{2, h, bad_alpha, beta, rho};
  expect(masw_dispersion_curve(nullptr, c.data(), 801, lam.data(), 30, &bm, MASW_PREC_FP64, 0, nullptr, ct.data(),
                               idx.data(), st.data(), cref.data()), E, "alpha <= beta");
  masw_model big{MASW_MAX_LAYERS + 1, h, alpha, beta, rho};
  expect(masw_dispersion_curve(nullptr, c.data(), 801, lam.data(), 30, &big, MASW_PREC_FP64, 0, nullptr, ct.data(),
                               idx.data(), st.data(), cref.data()), E, "too many layers");
  expect(masw_dispersion_curve(nullptr, c.data(), 801, lam.data(), 30, &m, masw_precision(7), 0, nullptr, ct.data(),
                               idx.data(), st.data(), cref.data()), E, "unknown precision");
  expect(masw_dispersion_curve(nullptr, c.data(), 801, lam.data(), 30, &m, MASW_PREC_FP64, 0x80u, nullptr,
                               ct.data(), idx.data(), st.data(), cref.data()), E, "unknown flag");
  expect(masw_dispersion_curve(nullptr, c.data(), 801, lam.data(), 30, &m, MASW_PREC_FP64, MASW_CHECK_NOISE,
                               nullptr, ct.data(), idx.data(), st.data(), cref.data()), E, "null context");
  expect(masw_dispersion_curve(nullptr, c.data(), 801, lam.data(), 30, &m, MASW_PREC_SPLIT, MASW_SEARCH_INERTIA,
                               nullptr, ct.data(), idx.data(), st.data(), cref.data()), E, "inertia with split");
  expect(masw_dispersion_curve_noalloc(nullptr, c.data(), 801, lam.data(), 30, &m, MASW_PREC_FP64, 0, nullptr,
                                       ct.data(), idx.data(), st.data(), cref.data()), E, "noalloc host pointers");
  expect(masw_dispersion_curve_noalloc(nullptr, c.data(), 1, lam.data(), 30, &m, MASW_PREC_FP64, MASW_DEVICE_PTRS,
                                       nullptr, ct.data(), idx.data(), st.data(), cref.data()), E, "noalloc short grid");
  expect(masw_dispersion_curve_noalloc(nullptr, c.data(), 801, lam.data(), 30, &big, MASW_PREC_FP64,
                                       MASW_DEVICE_PTRS, nullptr, ct.data(), idx.data(), st.data(), cref.data()), E,
         "noalloc too many layers");
  expect(masw_dispersion_curve_noalloc(nullptr, c.data(), 801, lam.data(), 30, &m, MASW_PREC_FP64,
                                       MASW_DEVICE_PTRS, nullptr, ct.data(), idx.data(), st.data(), cref.data()), E,
         "noalloc null context");

  // batch: offsets
  const int32_t loff[3] = {0, 2, 4}, woff_bad[3] = {0, 30, 20};
  const double h2[4] = {2.0, 4.0, 2.0, 4.0};
  double a2[6], b2[6], r2[6];
  for (int j = 0; j < 6; ++j) { a2[j] = alpha[j % 3]; b2[j] = beta[j % 3]; r2[j] = rho[j % 3]; }
  std::vector<double> lam2(60, 5.0);
  masw_batch b{2, loff, h2, a2, b2, r2, woff_bad, lam2.data()};
  masw_outputs o{ct.data(), idx.data(), st.data(), cref.data()};
  expect(masw_dispersion_batch(nullptr, c.data(), 801, &b, MASW_PREC_SPLIT, 0, nullptr, &o), E,
         "lambda_off decreasing");
  const int32_t woff[3] = {0, 15, 30};
  b.lambda_off = woff;
  b.n_models = 0;
  expect(masw_dispersion_batch(nullptr, c.data(), 801, &b, MASW_PREC_SPLIT, 0, nullptr, &o), E, "no models");

  // sign map, misfit, classification
  std::vector<int8_t> sig(30 * 801);
  expect(masw_sign_map(nullptr, c.data(), 801, lam.data(), 30, &bm, MASW_PREC_FP64, 0, nullptr, sig.data(),
                       nullptr), E, "sign map alpha <= beta");
  const double ce_bad[3] = {100.0, 0.0, 300.0};
  const int32_t moff[3] = {0, 2, 3};
  double mis[2];
  expect(masw_misfit(nullptr, 2, moff, ct.data(), ce_bad, 0, nullptr, mis), E, "misfit C_e <= 0");
  b.n_models = 2;
  std::vector<int32_t> pidx(30, 10), pcls(30);
  std::vector<double> psec(30);
  b.alpha = bad_alpha;  // model 0: alpha <= beta
  expect(masw_classify_picks(nullptr, c.data(), 801, &b, pidx.data(), 0, nullptr, pcls.data(), psec.data()), E,
         "classify alpha <= beta");
  b.alpha = a2;
  expect(masw_classify_picks(nullptr, c.data(), 801, &b, pidx.data(), 0x40u, nullptr, pcls.data(), psec.data()), E,
         "classify unknown flag");

  // serving without a server, stats and timing without a context
  uint64_t t = 0;
  expect(masw_submit(nullptr, c.data(), 801, lam.data(), 30, &m, MASW_PREC_FP64, 0, &t), E, "submit null context");
  expect(masw_submit(nullptr, c.data(), 801, lam.data(), 30, &m, MASW_PREC_FP64, MASW_DEVICE_PTRS, &t), E,
         "submit with a flag requests do not take");
  expect(masw_server_start(nullptr, nullptr), E, "server start null context");
  masw_stats s;
  expect(masw_get_stats(nullptr, &s), E, "stats null context");
  masw_timing tm;
  expect(masw_get_timing(nullptr, 0, &tm), E, "timing null context");
  ++checks;
  if (std::strcmp(masw_strerror(MASW_EINVAL), "invalid argument") != 0) ++failures;

  // no device here: creating a context fails cleanly
  masw_ctx* ctx = nullptr;
  const int rc = masw_create(0, size_t(1) << 20, &ctx);
  ++checks;
  if (rc == MASW_OK) {
    masw_destroy(ctx);  // a device is present after all: nothing to check
  } else if (rc != MASW_EDEVICE || ctx != nullptr) {
    ++failures;
    std::fprintf(stderr, "FAIL masw_create without a device: rc %d\n", rc);
  }
  masw_destroy(nullptr);

  std::printf("host sanitizer driver: %d checks, %d failures\n", checks, failures);
  return failures ? 1 : 0;
}
