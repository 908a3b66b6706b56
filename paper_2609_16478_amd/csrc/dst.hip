// Batched DST-I passes for gfx950.
//
// The subproblems of the augmented scheme are Dirichlet problems for the
// compact operator L_h, which the tensor sine basis diagonalises (the fast
// Poisson solver of Sec. 2.3 / Remark 2).  One pass transforms every pencil
// of an interior array along one axis:  X_k = sum_{m=1}^{N-1} x_m sin(pi k m / N).
//
// Per work-group, a tile of P pencils is staged in LDS.  Two real pencils a, b
// are packed as one complex sequence z = a + i b of length N (z_0 = 0), and the
// pair is transformed with ONE complex N-point FFT:
//   w_m = sin(pi m/N)(z_m + z_{N-m}) + (z_m - z_{N-m})/2,   W = FFT_N(w)
//   A_k = (W_k + conj W_{N-k})/2 (pencil a),  B_k = (W_k - conj W_{N-k})/(2i) (pencil b)
//   X_{2k} = -Im C_k,  X_1 = Re C_0 / 2,  X_{2k+1} = X_{2k-1} + Re C_k   (C = A or B)
// so a pencil of N-1 reals needs N/2 complex words of LDS -- the tile keeps
// 128 B row segments in the strided passes within the 160 KB LDS.  The odd
// outputs are a prefix sum (per-thread serial chunk + work-group offsets).
//
// The FFT is a Stockham autosort with radices 8/4/3/2, in place in LDS with
// register staging (all reads of a stage, barrier, all writes).  Twiddles
// come from a per-length table in global memory (L1/L2 resident).
//
// The fused middle pass (slowest axis) does forward DST, multiplies mode
// (k_x, k_y, k_z) by scale / lambda(k), and applies the DST again, before one
// store: lambda = sum_a s_a + sum_{a<b} (h_a^2 + h_b^2)/12 s_a s_b with
// s_a(k) = -(4/h_a^2) sin^2(k pi / (2 N_a)).
#include <atomic>
#include "common.h"

#include <cmath>
#include <cstdio>
#include <mutex>
#include <vector>

namespace ahoc {

namespace {

template <typename T> __device__ __forceinline__ cx<T> mk(T x, T y) {
  cx<T> r;
  r.x = x;
  r.y = y;
  return r;
}
template <typename V> __device__ __forceinline__ V cadd(V a, V b) {
  V r;
  r.x = a.x + b.x;
  r.y = a.y + b.y;
  return r;
}
template <typename V> __device__ __forceinline__ V csub(V a, V b) {
  V r;
  r.x = a.x - b.x;
  r.y = a.y - b.y;
  return r;
}
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  V r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
// multiply by -i
template <typename V> __device__ __forceinline__ V cmni(V a) {
  V r;
  r.x = a.y;
  r.y = -a.x;
  return r;
}

// Forward DFTs (kernel exp(-2 pi i / R)) of small radices, in registers.
template <typename T> __device__ __forceinline__ void dft2(cx<T>* a) {
  cx<T> t = a[0];
  a[0] = cadd(t, a[1]);
  a[1] = csub(t, a[1]);
}

template <typename T> __device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  cx<T> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = cmni(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <typename T> __device__ __forceinline__ void dft3(cx<T>* a) {
  const T h = T(0.86602540378443864676372317075294);  // sqrt(3)/2
  cx<T> s = cadd(a[1], a[2]);
  cx<T> d = csub(a[1], a[2]);
  cx<T> m = mk<T>(a[0].x - T(0.5) * s.x, a[0].y - T(0.5) * s.y);
  a[0] = cadd(a[0], s);
  a[1] = mk<T>(m.x + h * d.y, m.y - h * d.x);
  a[2] = mk<T>(m.x - h * d.y, m.y + h * d.x);
}

template <typename T> __device__ __forceinline__ void dft8(cx<T>* a) {
  const T c = T(0.70710678118654752440084436210485);
  dft4<T>(a[0], a[2], a[4], a[6]);
  dft4<T>(a[1], a[3], a[5], a[7]);
  // twiddle the odd half by exp(-2 pi i k / 8), k = 0..3
  cx<T> o1 = mk<T>(c * (a[3].x + a[3].y), c * (a[3].y - a[3].x));
  cx<T> o2 = cmni(a[5]);
  cx<T> o3 = mk<T>(c * (a[7].y - a[7].x), -c * (a[7].x + a[7].y));
  cx<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6], o0 = a[1];
  a[0] = cadd(e0, o0);
  a[4] = csub(e0, o0);
  a[1] = cadd(e1, o1);
  a[5] = csub(e1, o1);
  a[2] = cadd(e2, o2);
  a[6] = csub(e2, o2);
  a[3] = cadd(e3, o3);
  a[7] = csub(e3, o3);
}

template <typename T, int R> __device__ __forceinline__ void dft(cx<T>* a) {
  if constexpr (R == 2) dft2<T>(a);
  if constexpr (R == 3) dft3<T>(a);
  if constexpr (R == 4) dft4<T>(a[0], a[1], a[2], a[3]);
  if constexpr (R == 8) dft8<T>(a);
}

// One Stockham stage of radix R over a sequence of length N in LDS.
// Thread ts of the sequence owns butterflies j = ts + b*TPS, b < PPT/R.
template <typename T, int PPT, int R>
__device__ __forceinline__ void stage(cx<T>* seq, int ts, int TPS, int N, int Ns,
                                      const cx<T>* __restrict__ tw) {
  constexpr int NB = PPT / R;
  cx<T> v[NB][R];
  const int NR = N / R;
  const int tws = N / (Ns * R);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = ts + b * TPS;
#pragma unroll
    for (int r = 0; r < R; ++r) v[b][r] = seq[j + r * NR];
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = ts + b * TPS;
    const int k = j % Ns;
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], tw[r * k * tws]);
    }
    dft<T, R>(v[b]);
    const int base = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) seq[base + r * Ns] = v[b][r];
  }
  __syncthreads();
}

struct Plan {
  int N;
  int nrad;
  int rad[12];
};

// Forward DST-I of the pencil pair held in `seq` (positions 1..N-1, seq[0] = 0).
// On return seq[m] = (X^a_m, X^b_m), m = 1..N-1, seq[0] = 0.  With SCALE, mode m
// of pencil a (b) is multiplied by scale / (A.x + B.x s[m-1])  ((A.y, B.y) for b).
template <typename T, int PPT, bool SCALE>
__device__ __forceinline__ void dst1_lds(cx<T>* seq, cx<T>* tot, int ts, int TPS, const Plan& pl,
                                         const cx<T>* __restrict__ tw, const T* __restrict__ sn,
                                         cx<T> A, cx<T> B, const T* __restrict__ s_this, T scale) {
  const int N = pl.N;
  // (1) symmetric pre-weighting
#pragma unroll
  for (int i = 0; i < PPT / 2; ++i) {
    const int m = 1 + ts + i * TPS;
    const cx<T> z = seq[m], zr = seq[N - m];
    const T w = sn[m];
    const T sx = w * (z.x + zr.x), sy = w * (z.y + zr.y);
    const T dx = T(0.5) * (z.x - zr.x), dy = T(0.5) * (z.y - zr.y);
    seq[m] = mk<T>(sx + dx, sy + dy);
    seq[N - m] = mk<T>(sx - dx, sy - dy);
  }
  __syncthreads();
  // (2) complex FFT of length N
  int Ns = 1;
  for (int st = 0; st < pl.nrad; ++st) {
    const int R = pl.rad[st];
    if constexpr (PPT % 8 == 0) {
      if (R == 8) stage<T, PPT, 8>(seq, ts, TPS, N, Ns, tw);
    }
    if constexpr (PPT % 4 == 0) {
      if (R == 4) stage<T, PPT, 4>(seq, ts, TPS, N, Ns, tw);
    }
    if constexpr (PPT % 3 == 0) {
      if (R == 3) stage<T, PPT, 3>(seq, ts, TPS, N, Ns, tw);
    }
    if (R == 2) stage<T, PPT, 2>(seq, ts, TPS, N, Ns, tw);
    Ns *= R;
  }
  // (3) split the pair, even outputs directly, odd outputs by prefix sum
  constexpr int H = PPT / 2;
  const int k0 = ts * H;
  cx<T> pre[H], ev[H];
  T ax = 0, ay = 0;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const int k = k0 + i;
    const cx<T> w1 = seq[k];
    const cx<T> w2 = seq[k == 0 ? 0 : N - k];
    T ca = T(0.5) * (w1.x + w2.x), cb = T(0.5) * (w1.y + w2.y);
    if (k == 0) {
      ca *= T(0.5);
      cb *= T(0.5);
    }
    ax += ca;
    ay += cb;
    pre[i] = mk<T>(ax, ay);
    ev[i] = mk<T>(T(0.5) * (w2.y - w1.y), T(0.5) * (w1.x - w2.x));
  }
  tot[ts] = mk<T>(ax, ay);
  __syncthreads();
  T ox = 0, oy = 0;
  for (int t = 0; t < ts; ++t) {
    const cx<T> v = tot[t];
    ox += v.x;
    oy += v.y;
  }
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const int k = k0 + i;
    cx<T> e = (k == 0) ? mk<T>(0, 0) : ev[i];
    cx<T> o = mk<T>(pre[i].x + ox, pre[i].y + oy);
    if constexpr (SCALE) {
      if (k > 0) {
        const T s = s_this[2 * k - 1];
        e.x *= scale / (A.x + B.x * s);
        e.y *= scale / (A.y + B.y * s);
      }
      const T s = s_this[2 * k];
      o.x *= scale / (A.x + B.x * s);
      o.y *= scale / (A.y + B.y * s);
    }
    seq[2 * k] = e;
    seq[2 * k + 1] = o;
  }
  __syncthreads();
}

template <typename T> struct PassArgs {
  const T* in;
  T* out;
  Plan pl;
  const cx<T>* tw;
  const T* sn;
  long long outer;   // rows (inner == 1) or slabs
  long long inner;   // contiguous extent; 1 = contiguous pencils
  long long pitch;   // row stride of contiguous pencils
  long long ntile_inner;
  DstScale<T> fs;
};

template <typename T> constexpr int launch_cap() { return sizeof(T) == 8 ? 256 : 512; }

template <typename T, int PPT, bool FUSED>
__global__ void __launch_bounds__(launch_cap<T>()) k_dst_pass(PassArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem);
  const int N = a.pl.N;
  const int L = N - 1;
  const int ld = N + 1;
  const int TPS = N / PPT;
  const int nseq = blockDim.x / TPS;
  const int P = 2 * nseq;
  const int s = threadIdx.x / TPS;
  const int ts = threadIdx.x - s * TPS;
  cx<T>* seq = lds + s * ld;
  cx<T>* tot = lds + nseq * ld + s * TPS;
  T* ldsr = reinterpret_cast<T*>(lds);

  const bool rows = (a.inner == 1);
  long long base = 0, c0 = 0;
  int ncols = P;
  if (rows) {
    base = (long long)blockIdx.x * P;  // first row of the tile
    const long long left = a.outer - base;
    ncols = left < P ? (int)left : P;
  } else {
    const long long o = blockIdx.x / a.ntile_inner;
    c0 = (blockIdx.x - o * a.ntile_inner) * (long long)P;
    base = o * (long long)L * a.inner + c0;
    const long long left = a.inner - c0;
    ncols = left < P ? (int)left : P;
  }

  // ---- load the tile: pencil p -> sequence p/2, component p%2, positions 1..L.
  // Batches of U independent global loads per thread are issued before their
  // LDS writes, so each wave keeps many HBM requests in flight.
  constexpr int U = 16;
  if (rows) {
    const int per_row = (L + blockDim.x - 1) / blockDim.x;
    const int iters = P * per_row;
    for (int it0 = 0; it0 < iters; it0 += U) {
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int it = it0 + u;
        const int p = it / per_row;
        const int m = (it - p * per_row) * blockDim.x + threadIdx.x;
        v[u] = (it < iters && p < ncols && m < L) ? a.in[(base + p) * a.pitch + m] : T(0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int it = it0 + u;
        const int p = it / per_row;
        const int m = (it - p * per_row) * blockDim.x + threadIdx.x;
        if (it < iters && m < L) ldsr[2 * ((p >> 1) * ld + m + 1) + (p & 1)] = v[u];
      }
    }
  } else {
    const int lp = __builtin_ctz(P);
    const int total = P * L;
    for (int e0 = 0; e0 < total; e0 += U * blockDim.x) {
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * blockDim.x + threadIdx.x;
        const int c = e & (P - 1);
        const int m = e >> lp;
        v[u] = (e < total && c < ncols) ? a.in[base + (long long)m * a.inner + c] : T(0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * blockDim.x + threadIdx.x;
        const int c = e & (P - 1);
        const int m = e >> lp;
        if (e < total) ldsr[2 * ((c >> 1) * ld + m + 1) + (c & 1)] = v[u];
      }
    }
  }
  for (int q = threadIdx.x; q < nseq; q += blockDim.x) lds[q * ld] = mk<T>(0, 0);
  __syncthreads();

  cx<T> A = mk<T>(1, 1), B = mk<T>(0, 0);
  if constexpr (FUSED) {
    // columns of this pair, decoded into the other axes' mode indices
    const long long ca = c0 + 2 * s, cb = ca + 1;
    auto coef = [&](long long col, T& Ao, T& Bo) {
      const long long ib = col / a.fs.na;
      const long long ia = col - ib * a.fs.na;
      if (col >= a.inner || ia >= a.fs.nva) {
        Ao = 1;
        Bo = 0;
        return;
      }
      const T sa = a.fs.s_a[ia];
      const T sb = a.fs.s_b ? a.fs.s_b[ib] : T(0);
      Ao = sa + sb + a.fs.c_ab * sa * sb;
      Bo = T(1) + a.fs.c_ta * sa + a.fs.c_tb * sb;
      Ao += a.fs.a0 + a.fs.ka * sa + a.fs.kb * sb;  // v-equation shift (zero otherwise)
      Bo += a.fs.kt;
    };
    coef(ca, A.x, B.x);
    coef(cb, A.y, B.y);
    dst1_lds<T, PPT, true>(seq, tot, ts, TPS, a.pl, a.tw, a.sn, A, B, a.fs.s_this, a.fs.scale);
    dst1_lds<T, PPT, false>(seq, tot, ts, TPS, a.pl, a.tw, a.sn, A, B, nullptr, T(0));
  } else {
    dst1_lds<T, PPT, false>(seq, tot, ts, TPS, a.pl, a.tw, a.sn, A, B, nullptr, T(0));
  }

  // ---- store
  if (rows) {
    const int per_row = (L + blockDim.x - 1) / blockDim.x;
    const int iters = ncols * per_row;
#pragma unroll 4
    for (int it = 0; it < iters; ++it) {
      const int p = it / per_row;
      const int m = (it - p * per_row) * blockDim.x + threadIdx.x;
      if (m < L) a.out[(base + p) * a.pitch + m] = ldsr[2 * ((p >> 1) * ld + m + 1) + (p & 1)];
    }
  } else {
    const int lp = __builtin_ctz(P);
    const int total = P * L;
#pragma unroll 4
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
      const int c = e & (P - 1);
      const int m = e >> lp;
      if (c < ncols) a.out[base + (long long)m * a.inner + c] = ldsr[2 * ((c >> 1) * ld + m + 1) + (c & 1)];
    }
  }
}

void make_plan(int N, int ppt, Plan& pl) {
  pl.N = N;
  pl.nrad = 0;
  int m = N;
  const int cand[4] = {8, 4, 3, 2};
  for (int ci = 0; ci < 4; ++ci) {
    const int R = cand[ci];
    while (m % R == 0 && ppt % R == 0 && m > 1 && pl.nrad < 12) {
      pl.rad[pl.nrad++] = R;
      m /= R;
    }
  }
  if (m != 1) pl.nrad = -1;
}

template <typename T, int PPT, bool F> void set_lds_attr() {
  static std::once_flag once;
  std::call_once(once, [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dst_pass<T, PPT, F>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  });
}

template <typename T, int PPT>
int launch_ppt(const PassArgs<T>& a, bool fused, dim3 grid, dim3 block, size_t lds, hipStream_t st) {
  if (fused) {
    set_lds_attr<T, PPT, true>();
    hipLaunchKernelGGL((k_dst_pass<T, PPT, true>), grid, block, lds, st, a);
  } else {
    set_lds_attr<T, PPT, false>();
    hipLaunchKernelGGL((k_dst_pass<T, PPT, false>), grid, block, lds, st, a);
  }
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

}  // namespace

int dst_ppt(int N) {
  const int opts[5] = {32, 24, 16, 12, 8};
  for (int i = 0; i < 5; ++i) {
    if (N % opts[i] == 0) {
      Plan pl;
      make_plan(N, opts[i], pl);
      if (pl.nrad > 0) return opts[i];
    }
  }
  return 0;
}

bool dst_supported(int N) { return N >= 2 && N <= DST_MAX_N; }

int dev_alloc(const DevAlloc& a, void** p, size_t bytes) {
  if (bytes == 0) bytes = 8;
  *p = nullptr;
  if (a.alloc) {
    *p = a.alloc(bytes, a.ctx);
    if (!*p) {
      set_last_error("the caller's allocator returned NULL", "dev_alloc");
      return ST_NOMEM;
    }
    return ST_OK;
  }
  const hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    set_last_error(hipGetErrorString(e), "hipMalloc");
    (void)hipGetLastError();
    *p = nullptr;
    return ST_NOMEM;
  }
  return ST_OK;
}

void dev_free(const DevAlloc& a, void* p) {
  if (!p) return;
  if (a.alloc) {
    if (a.free) a.free(p, a.ctx);
    return;
  }
  (void)hipFree(p);
}

// Sequences (pencil pairs) per work-group: 128 B row segments for the strided
// passes where LDS allows, at least one wavefront, within the launch cap.
int dst_default_tile(int N, int elem_bytes) {
  const int ppt = dst_ppt(N);
  if (!ppt) return 0;
  const int tps = N / ppt;
  const int cap = elem_bytes == 8 ? 256 : 512;
  const int cxb = 2 * elem_bytes;
  int nseq = elem_bytes == 8 ? 8 : 16;
  while (nseq * tps < 64) nseq *= 2;
  while (nseq > 1 && (nseq * tps > cap || (size_t)(nseq * (N + 1) + nseq * tps) * cxb > 160 * 1024))
    nseq /= 2;
  if (nseq * tps > cap) return 0;
  return nseq;
}

template <typename T> int dst_tables_init(DstTables<T>& tb, int N, hipStream_t st, const DevAlloc* al) {
  dst_tables_free(tb);
  if (!dst_supported(N)) return ST_UNSUPPORTED;
  tb.al = al ? *al : DevAlloc();
  const int ppt = dst_ppt(N);
  const long double pi = 3.141592653589793238462643383279502884L;
  tb.N = N;
  tb.ppt = ppt;
  if (!ppt) {
    // no FFT plan: the direct pass reads one full period of sin(pi j / N); the integer
    // argument is reduced to [0, N] by the symmetries of the sine before evaluation
    std::vector<T> sn2(2 * (size_t)N);
    for (int j = 0; j < 2 * N; ++j) {
      const int r = j <= N ? j : 2 * N - j;
      const long double v = sinl(pi * (long double)(r <= N / 2 ? r : N - r) / (long double)N);
      sn2[j] = (T)(j <= N ? v : -v);
    }
    tb.nrad = 0;
    TRY_ST(dev_alloc(tb.al, reinterpret_cast<void**>(&tb.sn), sizeof(T) * 2 * (size_t)N));
    AHOC_HIP_TRY(hipMemcpyAsync(tb.sn, sn2.data(), sizeof(T) * 2 * (size_t)N, hipMemcpyHostToDevice, st));
    AHOC_HIP_TRY(hipStreamSynchronize(st));
  } else {
    Plan pl;
    make_plan(N, ppt, pl);
    tb.nrad = pl.nrad;
    for (int i = 0; i < pl.nrad; ++i) tb.rad[i] = pl.rad[i];
    std::vector<cx<T>> tw(N);
    std::vector<T> sn(N / 2 + 1);
    for (int k = 0; k < N; ++k) {
      const long double ang = 2.0L * pi * (long double)k / (long double)N;
      tw[k].x = (T)cosl(ang);
      tw[k].y = (T)(-sinl(ang));
    }
    for (int m = 0; m <= N / 2; ++m) sn[m] = (T)sinl(pi * (long double)m / (long double)N);
    TRY_ST(dev_alloc(tb.al, reinterpret_cast<void**>(&tb.tw), sizeof(cx<T>) * N));
    TRY_ST(dev_alloc(tb.al, reinterpret_cast<void**>(&tb.sn), sizeof(T) * (N / 2 + 1)));
    // stream-ordered uploads (no legacy-stream operation while other streams may be capturing)
    AHOC_HIP_TRY(hipMemcpyAsync(tb.tw, tw.data(), sizeof(cx<T>) * N, hipMemcpyHostToDevice, st));
    AHOC_HIP_TRY(hipMemcpyAsync(tb.sn, sn.data(), sizeof(T) * (N / 2 + 1), hipMemcpyHostToDevice, st));
    AHOC_HIP_TRY(hipStreamSynchronize(st));
  }
  if (dst_gemm_supported(N)) {
    const int rc = dst_gemm_table<T>(&tb.S, N, st, tb.al);
    if (rc != ST_OK) return rc;
  }
  return ST_OK;
}

template <typename T> int dst_plan_only(DstTables<T>& tb, int N) {
  const int ppt = dst_ppt(N);
  if (!ppt) return ST_UNSUPPORTED;
  Plan pl;
  make_plan(N, ppt, pl);
  tb.N = N;
  tb.ppt = ppt;
  tb.nrad = pl.nrad;
  for (int i = 0; i < pl.nrad; ++i) tb.rad[i] = pl.rad[i];
  return ST_OK;
}

template <typename T> void dst_tables_free(DstTables<T>& tb) {
  dev_free(tb.al, tb.tw);
  dev_free(tb.al, tb.sn);
  dev_free(tb.al, tb.S);
  tb.tw = nullptr;
  tb.sn = nullptr;
  tb.S = nullptr;
  tb.method[0] = tb.method[1] = -1;
  tb.N = 0;
}

// Process-wide kernel-family switch (a test and tuning hook, read at every pass; relaxed
// atomic so that setting it while other threads run passes is not a data race -- which
// family those passes use is then unspecified)
static std::atomic<int> g_variant_{0};
void dst_set_variant(int v) { g_variant_.store(v, std::memory_order_relaxed); }
int dst_get_variant() { return g_variant_.load(std::memory_order_relaxed); }

template <typename T>
int dst_pass(const DstTables<T>& tb, const T* in, T* out, long long outer, long long inner,
             long long pitch, const DstScale<T>* fused, int tile_seqs, hipStream_t st,
             const DstFaces<T>* faces) {
  const int N = tb.N;
  const int g_variant = dst_get_variant();
  if (inner == 1 && pitch < N - 1) return ST_INVALID;
  // plain passes: the kernel chosen at setup (or the matrix-core product where forced)
  if (!fused && !(faces && faces->mode) && tile_seqs <= 0) {
    const int k = inner == 1 ? 0 : 1;
    if (tb.S && (g_variant == 4 || (g_variant == 0 && tb.method[k] == DST_M_GEMM))) {
      const int rc = dst_gemm_pass<T>(tb.S, N, in, out, outer, inner, pitch, st);
      if (rc != ST_UNSUPPORTED) return rc;
    }
    if (g_variant == 0 && tb.method[k] == DST_M_TILE) tile_seqs = tb.tile[k];
  }
  if (g_variant != 1 && dst_fast_supported(N)) {
    const int rc = dst_fast_pass<T>(N, tb.tw, tb.sn, in, out, outer, inner, pitch, fused, tile_seqs, st, faces);
    if (rc != ST_UNSUPPORTED || g_variant == 2) return rc;
  }
  if (faces && faces->mode) return ST_UNSUPPORTED;  // face sums only in the specialised kernels
  const int ppt = tb.ppt;
  if (!ppt) {  // no FFT plan for this length: the direct sine sums
    if (!tb.sn) return ST_INVALID;
    return dst_direct_pass<T>(N, tb.sn, in, out, outer, inner, pitch, fused, st);
  }
  if (!tb.tw) return ST_INVALID;
  const int tps = N / ppt;
  const int nseq = tile_seqs > 0 ? tile_seqs : dst_default_tile(N, (int)sizeof(T));
  if (nseq <= 0 || (nseq & (nseq - 1))) return ST_INVALID;
  const int threads = nseq * tps;
  if (threads > launch_cap<T>() || threads < 1) return ST_UNSUPPORTED;
  const size_t lds = (size_t)(nseq * (N + 1) + threads) * sizeof(cx<T>);
  if (lds > 160 * 1024) return ST_UNSUPPORTED;
  if (fused && inner == 1) return ST_INVALID;
  PassArgs<T> a;
  a.in = in;
  a.out = out;
  a.pl.N = N;
  a.pl.nrad = tb.nrad;
  for (int i = 0; i < tb.nrad; ++i) a.pl.rad[i] = tb.rad[i];
  a.tw = tb.tw;
  a.sn = tb.sn;
  a.outer = outer;
  a.inner = inner;
  a.pitch = pitch;
  const long long P = 2LL * nseq;
  long long blocks;
  if (inner == 1) {
    a.ntile_inner = 1;
    blocks = (outer + P - 1) / P;
  } else {
    a.ntile_inner = (inner + P - 1) / P;
    blocks = outer * a.ntile_inner;
  }
  if (fused) a.fs = *fused;
  if (blocks <= 0) return ST_OK;
  if (blocks > 0x7fffffffLL) return ST_UNSUPPORTED;
  dim3 grid((unsigned)blocks), block((unsigned)threads);
  switch (ppt) {
    case 32: return launch_ppt<T, 32>(a, fused != nullptr, grid, block, lds, st);
    case 24: return launch_ppt<T, 24>(a, fused != nullptr, grid, block, lds, st);
    case 16: return launch_ppt<T, 16>(a, fused != nullptr, grid, block, lds, st);
    case 12: return launch_ppt<T, 12>(a, fused != nullptr, grid, block, lds, st);
    case 8: return launch_ppt<T, 8>(a, fused != nullptr, grid, block, lds, st);
    default: return ST_UNSUPPORTED;
  }
}

template int dst_tables_init<float>(DstTables<float>&, int, hipStream_t, const DevAlloc*);
template int dst_tables_init<double>(DstTables<double>&, int, hipStream_t, const DevAlloc*);
template int dst_plan_only<float>(DstTables<float>&, int);
template int dst_plan_only<double>(DstTables<double>&, int);
template void dst_tables_free<float>(DstTables<float>&);
template void dst_tables_free<double>(DstTables<double>&);
template int dst_pass<float>(const DstTables<float>&, const float*, float*, long long, long long,
                             long long, const DstScale<float>*, int, hipStream_t, const DstFaces<float>*);
template int dst_pass<double>(const DstTables<double>&, const double*, double*, long long,
                              long long, long long, const DstScale<double>*, int, hipStream_t,
                              const DstFaces<double>*);

}  // namespace ahoc
