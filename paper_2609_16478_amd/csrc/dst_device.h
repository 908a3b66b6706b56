// Device building blocks of the length-specialised DST-I kernels (gfx950): compile-time
// twiddles, in-register DFTs, Stockham stage plans, the paired-pencil post-processing
// (split + prefix sum) and pre-weighting, the tile load with pre-weighting and the tile
// store.  Shared by the single-pass kernels and the spectral lift / face-sum kernels.
#pragma once

#include "common.h"

#include <type_traits>

namespace ahoc {

// ---------------------------------------------------------------------------------
// compile-time trigonometry: exp(-2 pi i e / R) with exact integer octant reduction
// ---------------------------------------------------------------------------------
namespace ct {

constexpr double PI = 3.14159265358979323846264338327950288;

constexpr double sin_t(double x) {  // |x| <= pi/4
  double term = x, sum = x;
  const double x2 = x * x;
  for (int n = 1; n < 14; ++n) {
    term *= -x2 / ((2.0 * n) * (2.0 * n + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double cos_t(double x) {
  double term = 1.0, sum = 1.0;
  const double x2 = x * x;
  for (int n = 1; n < 14; ++n) {
    term *= -x2 / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}
// cos(2 pi e / R) and sin(2 pi e / R)
constexpr double cos2pi(long e, long R) {
  e %= R;
  if (e < 0) e += R;
  const long q = (4 * e + R / 2) / R;  // nearest quarter turn
  const double r = 2.0 * PI * (double)(4 * e - q * R) / (4.0 * R);
  switch (q & 3) {
    case 0: return cos_t(r);
    case 1: return -sin_t(r);
    case 2: return -cos_t(r);
    default: return sin_t(r);
  }
}
constexpr double sin2pi(long e, long R) {
  e %= R;
  if (e < 0) e += R;
  const long q = (4 * e + R / 2) / R;
  const double r = 2.0 * PI * (double)(4 * e - q * R) / (4.0 * R);
  switch (q & 3) {
    case 0: return sin_t(r);
    case 1: return cos_t(r);
    case 2: return -sin_t(r);
    default: return -cos_t(r);
  }
}

template <int R> struct Tw {
  double c[R > 0 ? R : 1];
  double s[R > 0 ? R : 1];  // -sin: forward kernel exp(-2 pi i e / R) = c + i s
  constexpr Tw() : c(), s() {
    for (int e = 0; e < R; ++e) {
      c[e] = cos2pi(e, R);
      s[e] = -sin2pi(e, R);
    }
  }
};

}  // namespace ct

namespace fast {

template <typename V> __device__ __forceinline__ V add(V a, V b) { V r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename V> __device__ __forceinline__ V sub(V a, V b) { V r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }

// a * exp(-2 pi i e / R), with the exactly trivial rotations folded
template <typename T, int R, int E> __device__ __forceinline__ cx<T> rot(cx<T> a) {
  constexpr int e = ((E % R) + R) % R;
  cx<T> r;
  if constexpr (e == 0) {
    return a;
  } else if constexpr (4 * e == R) {  // -i
    r.x = a.y;
    r.y = -a.x;
  } else if constexpr (2 * e == R) {  // -1
    r.x = -a.x;
    r.y = -a.y;
  } else if constexpr (4 * e == 3 * R) {  // +i
    r.x = -a.y;
    r.y = a.x;
  } else {
    constexpr ct::Tw<R> tw{};
    constexpr T c = (T)tw.c[e], s = (T)tw.s[e];
    r.x = a.x * c - a.y * s;
    r.y = a.x * s + a.y * c;
  }
  return r;
}

// In-register forward DFT of R points stored at a[OFF + STRIDE * k], k < R.
template <typename T, int R, int STRIDE = 1, int OFF = 0> struct DFT {
  static constexpr int F = (R % 4 == 0 && R > 4) ? 4 : ((R % 2 == 0 && R > 2) ? 2 : ((R % 3 == 0 && R > 3) ? 3 : R));
  static __device__ __forceinline__ void run(cx<T>* a) {
    if constexpr (R == 1) {
      return;
    } else if constexpr (R == 2) {
      cx<T> t = a[OFF];
      a[OFF] = add(t, a[OFF + STRIDE]);
      a[OFF + STRIDE] = sub(t, a[OFF + STRIDE]);
    } else if constexpr (R == 3) {
      const T h = T(0.86602540378443864676372317075294);
      cx<T> x0 = a[OFF], x1 = a[OFF + STRIDE], x2 = a[OFF + 2 * STRIDE];
      cx<T> s = add(x1, x2), d = sub(x1, x2);
      cx<T> m;
      m.x = x0.x - T(0.5) * s.x;
      m.y = x0.y - T(0.5) * s.y;
      a[OFF] = add(x0, s);
      a[OFF + STRIDE].x = m.x + h * d.y;
      a[OFF + STRIDE].y = m.y - h * d.x;
      a[OFF + 2 * STRIDE].x = m.x - h * d.y;
      a[OFF + 2 * STRIDE].y = m.y + h * d.x;
    } else if constexpr (R == 4) {
      cx<T> x0 = a[OFF], x1 = a[OFF + STRIDE], x2 = a[OFF + 2 * STRIDE], x3 = a[OFF + 3 * STRIDE];
      cx<T> t0 = add(x0, x2), t1 = sub(x0, x2), t2 = add(x1, x3), t3 = sub(x1, x3);
      cx<T> t3r;
      t3r.x = t3.y;
      t3r.y = -t3.x;
      a[OFF] = add(t0, t2);
      a[OFF + 2 * STRIDE] = sub(t0, t2);
      a[OFF + STRIDE] = add(t1, t3r);
      a[OFF + 3 * STRIDE] = sub(t1, t3r);
    } else {
      // R = F * G: G-point DFTs over the F interleaved subsequences, twiddle, F-point DFTs
      constexpr int G = R / F;
      cx<T> b[R];
#pragma unroll
      for (int n1 = 0; n1 < F; ++n1) {
#pragma unroll
        for (int n2 = 0; n2 < G; ++n2) b[n1 * G + n2] = a[OFF + STRIDE * (n1 + F * n2)];
      }
      unroll_sub<0>(b);
#pragma unroll
      for (int k2 = 0; k2 < G; ++k2) {
#pragma unroll
        for (int k1 = 0; k1 < F; ++k1) a[OFF + STRIDE * (k2 + G * k1)] = b[k1 * G + k2];
      }
    }
  }
  // b holds F rows of G: transform rows, twiddle, then transform the F-point columns
  template <int N1> static __device__ __forceinline__ void unroll_sub(cx<T>* b) {
    if constexpr (N1 < F) {
      DFT<T, R / F, 1, N1 * (R / F)>::run(b);
      twiddle_row<N1, 1>(b);
      unroll_sub<N1 + 1>(b);
    } else {
      cols<0>(b);
    }
  }
  template <int N1, int K2> static __device__ __forceinline__ void twiddle_row(cx<T>* b) {
    if constexpr (K2 < R / F) {
      b[N1 * (R / F) + K2] = rot<T, R, N1 * K2>(b[N1 * (R / F) + K2]);
      twiddle_row<N1, K2 + 1>(b);
    }
  }
  template <int K2> static __device__ __forceinline__ void cols(cx<T>* b) {
    if constexpr (K2 < R / F) {
      DFT<T, F, R / F, K2>::run(b);
      cols<K2 + 1>(b);
    }
  }
};

// Stage plans: radices per length (product N); PPT = points per thread (a
// multiple of every radix); TPS = N / PPT threads per pencil pair.
template <int N> struct Plan;
template <> struct Plan<32> { static constexpr int S = 2, R0 = 4, R1 = 8, R2 = 1, PPT = 8; };
template <> struct Plan<64> { static constexpr int S = 2, R0 = 8, R1 = 8, R2 = 1, PPT = 8; };
template <> struct Plan<96> { static constexpr int S = 2, R0 = 8, R1 = 12, R2 = 1, PPT = 24; };
template <> struct Plan<128> { static constexpr int S = 2, R0 = 8, R1 = 16, R2 = 1, PPT = 16; };
template <> struct Plan<192> { static constexpr int S = 3, R0 = 4, R1 = 4, R2 = 12, PPT = 12; };
template <> struct Plan<256> { static constexpr int S = 2, R0 = 16, R1 = 16, R2 = 1, PPT = 16; };
template <> struct Plan<384> { static constexpr int S = 3, R0 = 8, R1 = 4, R2 = 12, PPT = 24; };
template <> struct Plan<512> { static constexpr int S = 2, R0 = 16, R1 = 32, R2 = 1, PPT = 32; };
template <> struct Plan<768> { static constexpr int S = 3, R0 = 8, R1 = 8, R2 = 12, PPT = 24; };
template <> struct Plan<1024> { static constexpr int S = 2, R0 = 32, R1 = 32, R2 = 1, PPT = 32; };
template <> struct Plan<2048> { static constexpr int S = 3, R0 = 16, R1 = 8, R2 = 16, PPT = 16; };
template <> struct Plan<4096> { static constexpr int S = 3, R0 = 16, R1 = 16, R2 = 16, PPT = 16; };
// Row-pass plans: contiguous pencils need no wide tiles for coalescing, so the row pass
// trades a third stage for 16 points per thread: one wavefront per pencil pair and small
// work-groups, many of which share a compute unit and overlap their load and FFT phases.
template <int N> struct RowPlan : Plan<N> {};
template <> struct RowPlan<512> { static constexpr int S = 3, R0 = 16, R1 = 8, R2 = 4, PPT = 16; };
template <> struct RowPlan<1024> { static constexpr int S = 3, R0 = 16, R1 = 16, R2 = 4, PPT = 16; };
template <int N, bool ROWP> using PlanOf = std::conditional_t<ROWP, RowPlan<N>, Plan<N>>;

__device__ __forceinline__ constexpr int pad(int m) { return m + (m >> 5); }
template <int N> __host__ __device__ constexpr int seq_stride() {
  // padded length, made odd so consecutive sequences start in different banks
  return (N + (N >> 5) + 1) | 1;
}

// Padded offset of a compile-time displacement c from a padded base: pad(x + c) =
// pad(x) + poff(c) whenever x mod 32 + c mod 32 < 32 (no carry into the next 32-block) or
// c is a multiple of 32.  Then every LDS access of a stage is one base register plus an
// immediate offset.
__host__ __device__ constexpr int poff(int c) { return c + (c >> 5); }
__host__ __device__ constexpr bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// A wave-uniform global address held in scalar registers; accesses through it add a
// per-lane 32-bit byte offset, which is the global load/store form with a scalar base and a
// 32-bit vector offset (no per-lane 64-bit address arithmetic).
struct SBase {
  using gchar = __attribute__((address_space(1))) char;
  gchar* p;
  __device__ __forceinline__ explicit SBase(const void* q) {
    const unsigned long long v = reinterpret_cast<unsigned long long>(q);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    p = reinterpret_cast<gchar*>(((unsigned long long)hi << 32) | lo);
  }
  __device__ __forceinline__ SBase(gchar* q, long long d) : p(q + d) {}
  __device__ __forceinline__ SBase plus(long long d) const { return SBase(p, d); }
  // raw bits of a 4-, 8- or 16-byte value
  template <int B> struct Raw;
  template <typename V> using Bits = typename Raw<(int)sizeof(V)>::type;
  template <typename V> __device__ __forceinline__ V ld(unsigned off) const {
    static_assert(sizeof(V) == 4 || sizeof(V) == 8 || sizeof(V) == 16, "4, 8 or 16 bytes");
    const Bits<V> r = *reinterpret_cast<const __attribute__((address_space(1))) Bits<V>*>(p + off);
    return __builtin_bit_cast(V, r);
  }
  template <typename V> __device__ __forceinline__ void st(unsigned off, const V& v) const {
    static_assert(sizeof(V) == 4 || sizeof(V) == 8 || sizeof(V) == 16, "4, 8 or 16 bytes");
    *reinterpret_cast<__attribute__((address_space(1))) Bits<V>*>(p + off) = __builtin_bit_cast(Bits<V>, v);
  }
  // streaming (non-temporal) forms: data touched once, kept from displacing reused lines
  template <typename V> __device__ __forceinline__ V ld_nt(unsigned off) const {
    static_assert(sizeof(V) == 4 || sizeof(V) == 8 || sizeof(V) == 16, "4, 8 or 16 bytes");
    const Bits<V> r =
        __builtin_nontemporal_load(reinterpret_cast<const __attribute__((address_space(1))) Bits<V>*>(p + off));
    return __builtin_bit_cast(V, r);
  }
  template <typename V> __device__ __forceinline__ void st_nt(unsigned off, const V& v) const {
    static_assert(sizeof(V) == 4 || sizeof(V) == 8 || sizeof(V) == 16, "4, 8 or 16 bytes");
    __builtin_nontemporal_store(__builtin_bit_cast(Bits<V>, v),
                                reinterpret_cast<__attribute__((address_space(1))) Bits<V>*>(p + off));
  }
};
template <> struct SBase::Raw<4> { using type = unsigned; };
template <> struct SBase::Raw<8> { typedef unsigned type __attribute__((ext_vector_type(2))); };
template <> struct SBase::Raw<16> { typedef unsigned type __attribute__((ext_vector_type(4))); };


// Synchronisation of the LDS exchanges inside one pencil pair's transform.  When the TPS
// lanes of a pair lie in one wavefront (TPS <= 64, a power of two dividing 64) only that
// wavefront exchanges data: its LDS accesses complete in order, so a wavefront-scope fence
// (which keeps the compiler from moving accesses across it) is enough and the other
// wavefronts of the work-group run on.  Otherwise a work-group barrier.  Phases that read
// other pairs' data (tile loads and stores) keep their own work-group barriers.
template <int TPS> __device__ __forceinline__ void pair_sync() {
  if constexpr (TPS <= 64 && 64 % TPS == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// One Stockham stage (radix R, input blocks Ns) over the sequence in LDS.
template <typename T, int N, int R, int NS, int PPT>
__device__ __forceinline__ void stage(cx<T>* seq, int ts, const cx<T>* __restrict__ tw) {
  constexpr int TPS = N / PPT;
  constexpr int NB = PPT / R;
  constexpr int NR = N / R;
  constexpr int TWS = N / (NS * R);
  // reads at ts + b TPS + r NR: linear when both strides are multiples of 32
  constexpr bool RLIN = NR % 32 == 0 && (NB == 1 || TPS % 32 == 0);
  // writes at base + r NS, base = (j - k) R + k: base mod 32 = k < NS when R NS >= 32 (powers
  // of two), any when NS is a multiple of 32, a multiple of R when NS = 1 and R divides 32
  constexpr bool WLIN = is_pow2(R) && is_pow2(NS) && (NS % 32 == 0 || R * NS >= 32 || (NS == 1 && 32 % R == 0));
  cx<T> v[NB][R];
  if constexpr (RLIN) {
    const cx<T>* rb = seq + pad(ts);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = rb[poff(b * TPS + r * NR)];
    }
  } else {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = ts + b * TPS;
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = seq[pad(j + r * NR)];
    }
  }
  pair_sync<TPS>();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = ts + b * TPS;
    const int k = (NS == 1) ? 0 : j % NS;
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const cx<T> w = tw[r * k * TWS];
        const cx<T> x = v[b][r];
        v[b][r].x = x.x * w.x - x.y * w.y;
        v[b][r].y = x.x * w.y + x.y * w.x;
      }
    }
    DFT<T, R>::run(v[b]);
    const int base = (j - k) * R + k;
    if constexpr (WLIN) {
      cx<T>* wb = seq + pad(base);
#pragma unroll
      for (int r = 0; r < R; ++r) wb[poff(r * NS)] = v[b][r];
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) seq[pad(base + r * NS)] = v[b][r];
    }
  }
  pair_sync<TPS>();
}

template <typename T, int N, class P> __device__ __forceinline__ void fft(cx<T>* seq, int ts, const cx<T>* __restrict__ tw) {
  stage<T, N, P::R0, 1, P::PPT>(seq, ts, tw);
  stage<T, N, P::R1, P::R0, P::PPT>(seq, ts, tw);
  if constexpr (P::S == 3) stage<T, N, P::R2, P::R0 * P::R1, P::PPT>(seq, ts, tw);
}

// 1/x for the eigenvalue scaling: the hardware reciprocal (1 ulp) in FP32; in FP64 the
// hardware estimate refined by two Newton-Raphson steps r <- r + r (1 - x r), which keeps
// the error at the last-bit level without the full IEEE division sequence.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

// Split the pair and form the DST-I outputs in place (positions 1..N-1, 0 -> 0).
// With SCALE, output m of pencil a (b) is multiplied by scale / (A.x + B.x s[m-1]); with
// MSYM also by the weighting operator's symbol C.x + D.x s[m-1].
template <typename T, int N, class P, bool SCALE, bool MSYM = false>
__device__ __forceinline__ void post(cx<T>* seq, cx<T>* tot, int ts, cx<T> A, cx<T> B,
                                     const T* __restrict__ s_this, T scale, cx<T> C = cx<T>{},
                                     cx<T> D = cx<T>{}) {
  constexpr int PPT = P::PPT;
  constexpr int TPS = N / PPT;
  constexpr int H = PPT / 2;
  cx<T> ev[H], cc[H];
  // (a) mirrored reads, lanes on consecutive k
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const int k = ts + i * TPS;
    const cx<T> w1 = seq[pad(k)];
    const cx<T> w2 = seq[pad(k == 0 ? 0 : N - k)];
    T ca = T(0.5) * (w1.x + w2.x), cb = T(0.5) * (w1.y + w2.y);
    if (k == 0) {
      ca *= T(0.5);
      cb *= T(0.5);
    }
    cc[i].x = ca;
    cc[i].y = cb;
    ev[i].x = T(0.5) * (w2.y - w1.y);
    ev[i].y = T(0.5) * (w1.x - w2.x);
  }
  pair_sync<TPS>();
  // (b) even outputs in place, odd slots temporarily hold the increments c_k
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const int k = ts + i * TPS;
    cx<T> e = ev[i];
    if (k == 0) {
      e.x = 0;
      e.y = 0;
    }
    if constexpr (SCALE) {
      if (k > 0) {
        const T s = s_this[2 * k - 1];
        if constexpr (MSYM) {
          e.x *= scale * (C.x + D.x * s) * recip(A.x + B.x * s);
          e.y *= scale * (C.y + D.y * s) * recip(A.y + B.y * s);
        } else {
          e.x *= scale * recip(A.x + B.x * s);
          e.y *= scale * recip(A.y + B.y * s);
        }
      }
    }
    seq[pad(2 * k)] = e;
    seq[pad(2 * k + 1)] = cc[i];
  }
  pair_sync<TPS>();
  // (c) prefix sum: serial over this thread's contiguous chunk, then lane scan of totals
  const int k0 = ts * H;
  T ax = 0, ay = 0;
  cx<T> pre[H];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const cx<T> c = seq[pad(2 * (k0 + i) + 1)];
    ax += c.x;
    ay += c.y;
    pre[i].x = ax;
    pre[i].y = ay;
  }
  // segmented inclusive scan of the chunk totals over the TPS threads of this pair
  constexpr int W = TPS < 64 ? TPS : 64;
  T sx = ax, sy = ay;
  const int lane = ts & (W - 1);
#pragma unroll
  for (int d = 1; d < W; d <<= 1) {
    const T ox = __shfl_up(sx, d, W), oy = __shfl_up(sy, d, W);
    if (lane >= d) {
      sx += ox;
      sy += oy;
    }
  }
  T offx = sx - ax, offy = sy - ay;  // exclusive within the wave segment
  if constexpr (TPS > 64) {
    // combine the wave segments of this pair through LDS
    constexpr int NW = TPS / 64;
    const int wv = ts >> 6;
    if (lane == 63) {
      tot[wv].x = sx;
      tot[wv].y = sy;
    }
    __syncthreads();
    for (int q = 0; q < wv; ++q) {
      offx += tot[q].x;
      offy += tot[q].y;
    }
    (void)NW;
  }
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const int k = k0 + i;
    cx<T> o;
    o.x = pre[i].x + offx;
    o.y = pre[i].y + offy;
    if constexpr (SCALE) {
      const T s = s_this[2 * k];
      if constexpr (MSYM) {
        o.x *= scale * (C.x + D.x * s) * recip(A.x + B.x * s);
        o.y *= scale * (C.y + D.y * s) * recip(A.y + B.y * s);
      } else {
        o.x *= scale * recip(A.x + B.x * s);
        o.y *= scale * recip(A.y + B.y * s);
      }
    }
    seq[pad(2 * k + 1)] = o;
  }
  pair_sync<TPS>();
}

// Pre-weighting of a sequence already in LDS (second transform of the fused pass).
template <typename T, int N, class P>
__device__ __forceinline__ void pre_lds(cx<T>* seq, int ts, const T* __restrict__ sn) {
  constexpr int PPT = P::PPT;
  constexpr int TPS = N / PPT;
  constexpr bool LIN = TPS % 32 == 0;
  cx<T> z[PPT / 2], zr[PPT / 2];
  cx<T>* lo = seq + pad(1 + ts);
  cx<T>* hi = seq + pad(N - 1 - ts);
#pragma unroll
  for (int i = 0; i < PPT / 2; ++i) {
    const int m = 1 + ts + i * TPS;
    z[i] = LIN ? lo[poff(i * TPS)] : seq[pad(m)];
    zr[i] = LIN ? hi[-poff(i * TPS)] : seq[pad(N - m)];
  }
  pair_sync<TPS>();
#pragma unroll
  for (int i = 0; i < PPT / 2; ++i) {
    const int m = 1 + ts + i * TPS;
    const T w = sn[m];
    const T sx = w * (z[i].x + zr[i].x), sy = w * (z[i].y + zr[i].y);
    const T dx = T(0.5) * (z[i].x - zr[i].x), dy = T(0.5) * (z[i].y - zr[i].y);
    cx<T> o1, o2;
    o1.x = sx + dx;
    o1.y = sy + dy;
    o2.x = sx - dx;
    o2.y = sy - dy;
    if constexpr (LIN) {
      lo[poff(i * TPS)] = o1;
      hi[-poff(i * TPS)] = o2;
    } else {
      seq[pad(m)] = o1;
      seq[pad(N - m)] = o2;
    }
  }
  if (ts == 0) {
    cx<T> zz;
    zz.x = 0;
    zz.y = 0;
    seq[0] = zz;
  }
  pair_sync<TPS>();
}

template <typename T> struct Args {
  const T* in;
  T* out;
  const cx<T>* tw;
  const T* sn;
  long long outer, inner, pitch, ntile_inner;
  int lg_nseq;
  DstScale<T> fs;
  DstFaces<T> fc;
  DstGen<T> gn;  // face-layer spectra added after the scaling (U-solve with spectral M)
  int ntst;      // non-temporal loads and stores (arrays larger than the caches)
};

// Arrays of at least this size stream through the caches: their passes load and store
// with the non-temporal policy.  Smaller ones (batches of small instances) are re-read from
// the caches by the next pass, which the non-temporal policy would prevent.
constexpr double NT_STORE_MIN_BYTES = 256.0 * 1024 * 1024;

// sum over the TPS lanes of one pencil pair (all lanes receive the total)
template <typename T, int TPS>
__device__ __forceinline__ void seg_sum4(T& a, T& b, T& c, T& d, cx<T>* tot, int ts) {
  constexpr int W = TPS < 64 ? TPS : 64;
#pragma unroll
  for (int m = W / 2; m >= 1; m >>= 1) {
    a += __shfl_xor(a, m, W);
    b += __shfl_xor(b, m, W);
    c += __shfl_xor(c, m, W);
    d += __shfl_xor(d, m, W);
  }
  if constexpr (TPS > 64) {
    const int wv = ts >> 6;
    if ((ts & 63) == 0) {
      tot[2 * wv].x = a;
      tot[2 * wv].y = b;
      tot[2 * wv + 1].x = c;
      tot[2 * wv + 1].y = d;
    }
    __syncthreads();
    a = b = c = d = 0;
    for (int q = 0; q < TPS / 64; ++q) {
      a += tot[2 * q].x;
      b += tot[2 * q].y;
      c += tot[2 * q + 1].x;
      d += tot[2 * q + 1].y;
    }
    __syncthreads();
  }
}

// Work-group size cap: 16 points per thread leave room for 1024-thread (FP32) or 512-thread
// (FP64) groups in the single-transform passes; the fused pass holds more live state.
template <typename T, int N, bool FUSED, bool ROWP> constexpr int cap() {
  return PlanOf<N, ROWP>::PPT <= 16 && !FUSED ? (sizeof(T) == 8 ? 512 : 1024) : (sizeof(T) == 8 ? 256 : 512);
}


// Load nseq pencil pairs of a tile into LDS with the symmetric pre-weighting
// w_m = s_m (z_m + z_{N-m}) + (z_m - z_{N-m}) / 2 applied on the fly: each item (pair q,
// position m in 1..N/2) reads the mirrored positions m and N-m of both pencils.  Pencil
// a of pair q is column 2q of the tile, b is column 2q+1; element (column c, position m)
// sits at c * ps + (m - 1) * es.
template <typename T, int N, int U = 8>
__device__ __forceinline__ void load_pre(cx<T>* lds, const T* __restrict__ src, const T* __restrict__ sn,
                                         bool rows, int nseq, int lgq, int ncols, int es, int ps) {
  constexpr int HN = N / 2;
  constexpr int LDQ = seq_stride<N>();
  {
    const int items = nseq * HN;
    for (int i0 = 0; i0 < items; i0 += U * (int)blockDim.x) {
      T xa[U], xb[U], ya[U], yb[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int it = i0 + u * blockDim.x + threadIdx.x;
        int q, m;
        if (rows) {
          q = it / HN;
          m = 1 + (it - q * HN);
        } else {
          q = it & (nseq - 1);
          m = 1 + (it >> lgq);
        }
        const bool ok = it < items;
        const int pa = 2 * q;
        const bool oka = ok && pa < ncols, okb = ok && pa + 1 < ncols;
        const int o1 = pa * ps + (m - 1) * es;       // pencil a, position m
        const int o2 = pa * ps + (N - m - 1) * es;   // pencil a, position N - m
        xa[u] = oka ? src[o1] : T(0);
        xb[u] = okb ? src[o1 + ps] : T(0);
        ya[u] = (oka && m < HN) ? src[o2] : T(0);
        yb[u] = (okb && m < HN) ? src[o2 + ps] : T(0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int it = i0 + u * blockDim.x + threadIdx.x;
        if (it < items) {
          int q, m;
          if (rows) {
            q = it / HN;
            m = 1 + (it - q * HN);
          } else {
            q = it & (nseq - 1);
            m = 1 + (it >> lgq);
          }
          const T w = sn[m];
          cx<T>* sq = lds + q * LDQ;
          if (m < HN) {
            const T sx = w * (xa[u] + ya[u]), sy = w * (xb[u] + yb[u]);
            const T dx = T(0.5) * (xa[u] - ya[u]), dy = T(0.5) * (xb[u] - yb[u]);
            cx<T> o1, o2;
            o1.x = sx + dx;
            o1.y = sy + dy;
            o2.x = sx - dx;
            o2.y = sy - dy;
            sq[pad(m)] = o1;
            sq[pad(N - m)] = o2;
          } else {  // m = N/2 pairs with itself: w = 2 z
            cx<T> o;
            o.x = T(2) * xa[u];
            o.y = T(2) * xb[u];
            sq[pad(m)] = o;
          }
        }
      }
    }
    if (threadIdx.x < nseq) {
      cx<T> zz;
      zz.x = 0;
      zz.y = 0;
      lds[threadIdx.x * LDQ] = zz;
    }
  }
}

// Store the N-1 outputs of each pencil pair from LDS (layout as in load_pre).
template <typename T, int N>
__device__ __forceinline__ void store_tile(const cx<T>* lds, T* __restrict__ dst, bool rows, int nseq, int lgq,
                                           int ncols, int es, int ps) {
  constexpr int L = N - 1;
  constexpr int LDQ = seq_stride<N>();
  const int items = nseq * L;
#pragma unroll 4
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    int q, m;
    if (rows) {
      q = it / L;
      m = 1 + (it - q * L);
    } else {
      q = it & (nseq - 1);
      m = 1 + (it >> lgq);
    }
    const cx<T> v = lds[q * LDQ + pad(m)];
    const int pa = 2 * q;
    const int o = pa * ps + (m - 1) * es;
    if (pa < ncols) dst[o] = v.x;
    if (pa + 1 < ncols) dst[o + ps] = v.y;
  }
}

}  // namespace fast
}  // namespace ahoc
