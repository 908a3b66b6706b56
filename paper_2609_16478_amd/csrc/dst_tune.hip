// Setup-time choice of the kernel for the plain DST-I passes of an operator.
//
// For a pass shape (precision, N, outer, inner, pitch) the candidates are timed on the
// device with HIP events and the fastest is kept:
//   DST_M_DEFAULT  the default FFT kernel (row kernel or persistent pipelined strided kernel),
//   DST_M_TILE     the one-tile FFT kernel with half, the default and twice the default tile
//                  of pencil pairs per work-group (for N = 512, 1024 also another radix plan:
//                  32 points per thread instead of 16),
//   DST_M_GEMM     the matrix-core products (even N <= 128).
// Passes over arrays of NT_STORE_MIN_BYTES or more skip the one-tile kernels (and, with no other
// candidate, keep the default kernel untimed).  Candidates that cannot launch (LDS, thread or
// length limits) are skipped.  The first
// timing of a shape is kept for the process, so every handle with that shape runs the same
// kernels and gives bit-identical results.
#include "common.h"
#include "dst_device.h"

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

namespace ahoc {

namespace {

struct Tuned {
  int method, tile;
  double t_default_us, t_gemm_us, t_best_us;
};
std::mutex g_mu;
std::map<std::tuple<int, int, long long, long long, long long>, Tuned> g_tuned;

}  // namespace

template <typename T>
int dst_autotune(DstTables<T>& tb, T* buf, long long outer, long long inner, long long pitch, hipStream_t st) {
  const int kind = inner == 1 ? 0 : 1;
  tb.method[kind] = -1;
  tb.tile[kind] = 0;
  tb.t_default_us[kind] = tb.t_gemm_us[kind] = tb.t_best_us[kind] = -1.0;
  if (dst_get_variant() != 0 || outer <= 0 || tb.N < 2) return ST_OK;
  const auto key = std::make_tuple((int)sizeof(T), tb.N, outer, inner, inner == 1 ? pitch : 0LL);
  auto apply = [&](const Tuned& r) {
    tb.method[kind] = r.method;
    tb.tile[kind] = r.tile;
    tb.t_default_us[kind] = r.t_default_us;
    tb.t_gemm_us[kind] = r.t_gemm_us;
    tb.t_best_us[kind] = r.t_best_us;
  };
  {
    std::lock_guard<std::mutex> lk(g_mu);
    const auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      apply(it->second);
      return ST_OK;
    }
  }
  const int N = tb.N, L = N - 1;
  const long long extent = inner == 1 ? (outer - 1) * pitch + L : outer * (long long)L * inner;
  struct Cand {
    int method, tile;
  };
  std::vector<Cand> cands{{DST_M_DEFAULT, 0}};
  if (tb.S) cands.push_back({DST_M_GEMM, 0});
  // arrays beyond the caches: the persistent kernels, which overlap the next tile's loads
  // with the current transform, beat the one-tile kernels on every measured shape, so only
  // cache-resident passes time them
  const bool big = (double)extent * sizeof(T) >= fast::NT_STORE_MIN_BYTES;
  if (!big && dst_fast_supported(N)) {
    const int d = dst_fast_tile(N, (int)sizeof(T), inner == 1 ? DST_PASS_ROWS : DST_PASS_STRIDED);
    for (int t : {d / 2, d, 2 * d})
      if (t >= 1 && (t & (t - 1)) == 0) cands.push_back({DST_M_TILE, t});
  }
  if (cands.size() == 1) return ST_OK;  // nothing to choose: the default kernel, untimed
  // zeros: the timings do not depend on the values, and repeated transforms stay finite
  AHOC_HIP_TRY(hipMemsetAsync(buf, 0, sizeof(T) * (size_t)extent, st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  AHOC_HIP_TRY(hipEventCreate(&e0));
  const hipError_t he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    (void)hipEventDestroy(e0);
    set_last_error(hipGetErrorString(he), "dst_autotune");
    return ST_HIP;
  }
  constexpr int REPS = 5;
  Tuned r{-1, 0, -1.0, -1.0, -1.0};
  int rc = ST_OK;
  for (const Cand& c : cands) {
    auto launch = [&]() -> int {
      switch (c.method) {
        case DST_M_GEMM: return dst_gemm_pass<T>(tb.S, N, buf, buf, outer, inner, pitch, st);
        case DST_M_TILE:
          return dst_fast_pass<T>(N, tb.tw, tb.sn, buf, buf, outer, inner, pitch, nullptr, c.tile, st);
        default: {
          const int m = tb.method[kind];
          tb.method[kind] = -1;  // dst_pass takes its default kernel
          const int q = dst_pass<T>(tb, buf, buf, outer, inner, pitch, nullptr, 0, st);
          tb.method[kind] = m;
          return q;
        }
      }
    };
    int q = launch();  // untimed warm-up; an unsupported configuration is skipped
    if (q == ST_UNSUPPORTED) continue;
    if (q != ST_OK) {
      rc = q;
      break;
    }
    if (hipEventRecord(e0, st) != hipSuccess) {
      rc = ST_HIP;
      break;
    }
    for (int i = 0; i < REPS && q == ST_OK; ++i) q = launch();
    float ms = 0.f;
    if (q != ST_OK) {
      rc = q;
      break;
    }
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      rc = ST_HIP;
      break;
    }
    const double us = 1e3 * ms / REPS;
    if (c.method == DST_M_DEFAULT) r.t_default_us = us;
    if (c.method == DST_M_GEMM) r.t_gemm_us = us;
    if (r.method < 0 || us < r.t_best_us) {
      r.method = c.method;
      r.tile = c.tile;
      r.t_best_us = us;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == ST_HIP) set_last_error("event timing failed", "dst_autotune");
  if (rc != ST_OK) return rc;
  if (r.method < 0) return ST_OK;  // nothing launched: keep the defaults
  {
    // a concurrent setup of the same shape may have stored its timing first: keep that one
    std::lock_guard<std::mutex> lk(g_mu);
    r = g_tuned.emplace(key, r).first->second;
  }
  apply(r);
  return ST_OK;
}

template int dst_autotune<float>(DstTables<float>&, float*, long long, long long, long long, hipStream_t);
template int dst_autotune<double>(DstTables<double>&, double*, long long, long long, long long, hipStream_t);

}  // namespace ahoc
