// Direct DST-I pass for transform lengths without a radix-2/3 FFT plan (gfx950).
//
// X_k = sum_{m=1}^{N-1} x_m sin(pi k m / N), k = 1..N-1, evaluated as written: O(N) work
// per output, with sin(pi j / N) read from a one-period table (index k m mod 2N, advanced
// incrementally).  It gives every grid length from the one-sided formula's minimum
// (N_a >= 4, Sec. 2.2) upward a pass with the same layouts as the FFT kernels: rows
// (contiguous pencils, `pitch` apart) or strided pencils [outer][L][inner].  The fused
// form (slowest axis of a Poisson solve) transforms, multiplies mode k of column c by
// scale / (A_c + B_c s_this[k-1]) -- the compact Laplacian's eigenvalue, Sec. 2.3 -- and
// transforms back before one store.
//
// A work-group stages a tile of P pencils in LDS (reads complete before any write, so the
// pass may run in place), then each thread forms outputs of one pencil at a time.
#include "common.h"

#include <mutex>

namespace ahoc {

namespace {

template <typename T> struct DirectArgs {
  const T* in;
  T* out;
  const T* sn2;       // sin(pi j / N), j = 0..2N-1
  int N;
  int P;              // pencils per work-group
  long long outer, inner, pitch;
  long long ntile_inner;
  bool fused;
  DstScale<T> fs;
};

// y_k = sum_m x_m sin(pi k m / N) for k = 1..L over the pencils of the tile held in `x`
// (pencil p at x + p * L), into y (same layout); threads take (p, k) with k fastest.
template <typename T>
__device__ void direct_sums(const T* x, T* y, int P, int L, int N, const T* __restrict__ sn2) {
  const int two_n = 2 * N;
  for (int e = threadIdx.x; e < P * L; e += blockDim.x) {
    const int p = e / L;
    const int k = e - p * L + 1;
    const T* xp = x + (long long)p * L;
    T acc = 0;
    int idx = 0;
    for (int m = 1; m <= L; ++m) {
      idx += k;
      if (idx >= two_n) idx -= two_n;
      acc += xp[m - 1] * sn2[idx];
    }
    y[e] = acc;
  }
}

template <typename T> __global__ void __launch_bounds__(256) k_dst_direct(DirectArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* x = reinterpret_cast<T*>(smem);
  const int L = a.N - 1;
  const int P = a.P;
  T* y = x + (long long)P * L;
  const bool rows = a.inner == 1;
  long long base, c0 = 0;
  int ncols;
  if (rows) {
    base = (long long)blockIdx.x * P;
    const long long left = a.outer - base;
    ncols = left < P ? (int)left : P;
  } else {
    const long long o = blockIdx.x / a.ntile_inner;
    c0 = (blockIdx.x - o * a.ntile_inner) * (long long)P;
    base = o * (long long)L * a.inner + c0;
    const long long left = a.inner - c0;
    ncols = left < P ? (int)left : P;
  }
  // load: rows with m fastest, strided pencils with the column fastest (coalesced)
  for (int e = threadIdx.x; e < P * L; e += blockDim.x) {
    int p, m;
    if (rows) {
      p = e / L;
      m = e - p * L;
    } else {
      m = e / P;
      p = e - m * P;
    }
    T v = 0;
    if (p < ncols) v = rows ? a.in[(base + p) * a.pitch + m] : a.in[base + (long long)m * a.inner + p];
    x[p * L + m] = v;
  }
  __syncthreads();
  T* res = y;
  if (a.fused) {
    direct_sums<T>(x, y, P, L, a.N, a.sn2);
    __syncthreads();
    for (int e = threadIdx.x; e < P * L; e += blockDim.x) {
      const int p = e / L;
      const int k = e - p * L + 1;
      const long long col = c0 + p;
      const long long ib = col / a.fs.na;
      const long long ia = col - ib * a.fs.na;
      T A = 1, B = 0;
      if (col < a.inner && ia < a.fs.nva) {
        const T sa = a.fs.s_a[ia];
        const T sb = a.fs.s_b ? a.fs.s_b[ib] : T(0);
        A = sa + sb + a.fs.c_ab * sa * sb + a.fs.a0 + a.fs.ka * sa + a.fs.kb * sb;
        B = T(1) + a.fs.c_ta * sa + a.fs.c_tb * sb + a.fs.kt;
      }
      y[e] *= a.fs.scale / (A + B * a.fs.s_this[k - 1]);
    }
    __syncthreads();
    direct_sums<T>(y, x, P, L, a.N, a.sn2);
    __syncthreads();
    res = x;
  } else {
    direct_sums<T>(x, y, P, L, a.N, a.sn2);
    __syncthreads();
  }
  for (int e = threadIdx.x; e < P * L; e += blockDim.x) {
    int p, k;
    if (rows) {
      p = e / L;
      k = e - p * L;
    } else {
      k = e / P;
      p = e - k * P;
    }
    if (p >= ncols) continue;
    const T v = res[p * L + k];
    if (rows) a.out[(base + p) * a.pitch + k] = v;
    else a.out[base + (long long)k * a.inner + p] = v;
  }
}

constexpr size_t DIRECT_LDS_MAX = 160 * 1024;

template <typename T> void set_direct_lds_attr() {
  static std::once_flag once;
  std::call_once(once, [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dst_direct<T>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)DIRECT_LDS_MAX);
  });
}

}  // namespace

template <typename T>
int dst_direct_pass(int N, const T* sn2, const T* in, T* out, long long outer, long long inner, long long pitch,
                    const DstScale<T>* fused, hipStream_t st) {
  if (N < 2 || N > DST_MAX_N || !sn2 || !in || !out || outer < 0 || inner < 1) return ST_INVALID;
  const int L = N - 1;
  if (inner == 1 && (pitch < L || fused)) return ST_INVALID;
  if (outer == 0) return ST_OK;
  const size_t per = (size_t)L * sizeof(T) * 2;  // x and y of one pencil
  int P = (int)std::min<size_t>(64, std::max<size_t>(1, (48 * 1024) / per));
  if ((size_t)P * per > DIRECT_LDS_MAX) return ST_UNSUPPORTED;
  DirectArgs<T> a;
  a.in = in;
  a.out = out;
  a.sn2 = sn2;
  a.N = N;
  a.P = P;
  a.outer = outer;
  a.inner = inner;
  a.pitch = pitch;
  a.fused = fused != nullptr;
  if (fused) a.fs = *fused;
  long long blocks;
  if (inner == 1) {
    a.ntile_inner = 1;
    blocks = (outer + P - 1) / P;
  } else {
    a.ntile_inner = (inner + P - 1) / P;
    blocks = outer * a.ntile_inner;
  }
  if (blocks > 0x7fffffffLL) return ST_UNSUPPORTED;
  const size_t lds = (size_t)P * per;
  if (lds > 64 * 1024) set_direct_lds_attr<T>();
  hipLaunchKernelGGL(k_dst_direct<T>, dim3((unsigned)blocks), dim3(256), lds, st, a);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

template int dst_direct_pass<float>(int, const float*, const float*, float*, long long, long long, long long,
                                    const DstScale<float>*, hipStream_t);
template int dst_direct_pass<double>(int, const double*, const double*, double*, long long, long long, long long,
                                     const DstScale<double>*, hipStream_t);

}  // namespace ahoc
