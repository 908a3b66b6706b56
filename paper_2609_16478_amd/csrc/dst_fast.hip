// DST-I pass kernels specialised on the transform length N (gfx950).
//
// Same transform as the generic kernel in dst.hip (two real pencils packed in
// one complex N-point FFT, symmetric pre-weighting, split + prefix sum for the
// odd outputs), organised for the instruction and LDS budget of CDNA4:
//
//  * the FFT is 2-3 Stockham stages of radix 8..32 computed in registers; the
//    in-register DFTs are unrolled with compile-time twiddle constants, and the
//    length, strides and stage twiddle indices are compile-time expressions;
//  * the symmetric pre-weighting w_m = s_m (z_m + z_{N-m}) + (z_m - z_{N-m})/2
//    is applied while the tile is read from HBM (each work item loads the
//    mirrored pair m, N-m of both pencils), so it costs no LDS round trip;
//  * LDS indices are padded by one complex word every 32 (pos + pos/32) and the
//    per-sequence stride is odd in banks, so the stage writes of stride R, the
//    mirrored post-processing reads and the chunked prefix sum are free of
//    bank conflicts;
//  * the odd outputs' prefix sum runs as a serial sum over a contiguous chunk
//    per thread plus a segmented lane scan of the chunk totals (shuffles).
#include <atomic>
#include "dst_device.h"

#include <mutex>

namespace ahoc {

namespace fast {

template <typename T, int N, bool FUSED, int FACES, bool ROWP>
__global__ void __launch_bounds__((cap<T, N, FUSED, ROWP>())) k_dst_fast(Args<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  using PL = PlanOf<N, ROWP>;
  constexpr int PPT = PL::PPT;
  constexpr int TPS = N / PPT;
  constexpr int L = N - 1;
  constexpr int LDQ = seq_stride<N>();
  constexpr int HN = N / 2;
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem);
  const int nseq = blockDim.x / TPS;
  const int lgq = a.lg_nseq;
  const int s = threadIdx.x / TPS;
  const int ts = threadIdx.x - s * TPS;
  constexpr int NTOT = 2 * (TPS / 64 > 0 ? TPS / 64 : 1);  // per pair: scan / face partials
  cx<T>* seq = lds + s * LDQ;
  cx<T>* tot = lds + nseq * LDQ + s * NTOT;
  const int P = 2 * nseq;

  // The tile's first element (uniform 64-bit base); per-lane offsets below are 32-bit.
  const bool rows = (a.inner == 1);
  long long base = 0, c0 = 0;
  int ncols = P;
  int es, ps;  // element stride along a pencil, stride between pencils
  if (rows) {
    const long long row0 = (long long)blockIdx.x * P;
    base = row0 * a.pitch;
    const long long left = a.outer - row0;
    ncols = left < P ? (int)left : P;
    es = 1;
    ps = (int)a.pitch;
  } else {
    const long long o = blockIdx.x / a.ntile_inner;
    c0 = (blockIdx.x - o * a.ntile_inner) * (long long)P;
    base = o * (long long)L * a.inner + c0;
    const long long left = a.inner - c0;
    ncols = left < P ? (int)left : P;
    es = (int)a.inner;
    ps = 1;
  }
  const T* __restrict__ src = a.in + base;
  T* __restrict__ dst = a.out + base;

  // ---- load + pre-weighting
  load_pre<T, N>(lds, src, a.sn, rows, nseq, lgq, ncols, es, ps);
  __syncthreads();

  cx<T> A, B;
  A.x = A.y = T(1);
  B.x = B.y = T(0);
  fft<T, N, PL>(seq, ts, a.tw);
  if constexpr (FUSED) {
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
    post<T, N, PL, true>(seq, tot, ts, A, B, a.fs.s_this, a.fs.scale);
    if constexpr (FACES == 1) {
      // face sums of the scaled spectrum along this axis, per column; the scaled spectrum
      // itself is the output (no inverse transform)
      T la = 0, ha = 0, lb = 0, hb = 0;
#pragma unroll
      for (int i = 0; i < PPT; ++i) {
        const int m = 1 + ts + i * TPS;
        if (m < N) {
          const cx<T> v = seq[pad(m)];
          const T wl = a.fc.w[m - 1], wh = a.fc.w[L + m - 1];
          la += v.x * wl;
          ha += v.x * wh;
          lb += v.y * wl;
          hb += v.y * wh;
        }
      }
      seg_sum4<T, TPS>(la, ha, lb, hb, tot, ts);
      if (ts == 0) {
        T* fo = a.fc.out + (blockIdx.x / a.ntile_inner) * a.fc.slab;
        if (ca < a.inner) {
          fo[ca] = la;
          fo[a.fc.plane + ca] = ha;
        }
        if (cb < a.inner) {
          fo[cb] = lb;
          fo[a.fc.plane + cb] = hb;
        }
      }
    }
    if constexpr (FACES == 0) {
      pre_lds<T, N, PL>(seq, ts, a.sn);
      fft<T, N, PL>(seq, ts, a.tw);
      post<T, N, PL, false>(seq, tot, ts, A, B, nullptr, T(0));
    }
  } else {
    post<T, N, PL, false>(seq, tot, ts, A, B, nullptr, T(0));
  }

  __syncthreads();  // the store reads other pairs' sequences
  store_tile<T, N>(lds, dst, rows, nseq, lgq, ncols, es, ps);
}

template <typename T, int N, bool F, int FC, bool RP> void set_attr() {
  static std::once_flag once;
  std::call_once(once, [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dst_fast<T, N, F, FC, RP>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  });
}

template <typename T, int N, bool F, int FC, bool RP>
int launch_one(const Args<T>& a, int nseq, hipStream_t st) {
  constexpr int TPS = N / PlanOf<N, RP>::PPT;
  const int threads = nseq * TPS;
  if (threads > cap<T, N, F, RP>() || threads % 64 != 0) return ST_UNSUPPORTED;
  const int ntot = nseq * 2 * (TPS / 64 > 0 ? TPS / 64 : 1);
  const size_t lds = (size_t)(nseq * seq_stride<N>() + ntot) * sizeof(cx<T>);
  if (lds > 160 * 1024) return ST_UNSUPPORTED;
  const long long P = 2LL * nseq;
  const long long blocks = a.inner == 1 ? (a.outer + P - 1) / P : a.outer * a.ntile_inner;
  if (blocks <= 0) return ST_OK;
  if (blocks > 0x7fffffffLL) return ST_UNSUPPORTED;
  set_attr<T, N, F, FC, RP>();
  hipLaunchKernelGGL((k_dst_fast<T, N, F, FC, RP>), dim3((unsigned)blocks), dim3(threads), lds, st, a);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

template <int N> constexpr bool has_row_plan() { return N == 512 || N == 1024; }

template <typename T, int N>
int launch(const Args<T>& a, int kind, int nseq, hipStream_t st) {
  if (kind == DST_PASS_FUSED) {
    if (a.fc.mode == 1) return launch_one<T, N, true, 1, false>(a, nseq, st);
    if (a.fc.mode == 0) return launch_one<T, N, true, 0, false>(a, nseq, st);
    return ST_INVALID;
  }
  if (a.fc.mode != 0) return ST_INVALID;
  if constexpr (has_row_plan<N>()) {
    if (kind == DST_PASS_ROWS) return launch_one<T, N, false, 0, true>(a, nseq, st);
  }
  return launch_one<T, N, false, 0, false>(a, nseq, st);
}

}  // namespace fast

bool dst_fast_supported(int N) {
  switch (N) {
    case 32: case 64: case 96: case 128: case 192: case 256: case 384: case 512: case 768:
    case 1024: case 2048: case 4096:
      return true;
    default:
      return false;
  }
}

// Threads per pencil pair of the plan a pass of this kind uses.
static int fast_tps(int N, int kind) {
  const bool rp = kind == DST_PASS_ROWS;
  switch (N) {
    case 32: return 32 / fast::Plan<32>::PPT;
    case 64: return 64 / fast::Plan<64>::PPT;
    case 96: return 96 / fast::Plan<96>::PPT;
    case 128: return 128 / fast::Plan<128>::PPT;
    case 192: return 192 / fast::Plan<192>::PPT;
    case 256: return 256 / fast::Plan<256>::PPT;
    case 384: return 384 / fast::Plan<384>::PPT;
    case 512: return 512 / (rp ? fast::RowPlan<512>::PPT : fast::Plan<512>::PPT);
    case 768: return 768 / fast::Plan<768>::PPT;
    case 1024: return 1024 / (rp ? fast::RowPlan<1024>::PPT : fast::Plan<1024>::PPT);
    case 2048: return 2048 / fast::Plan<2048>::PPT;
    case 4096: return 4096 / fast::Plan<4096>::PPT;
    default: return 0;
  }
}

// Process-wide tile override per pass kind and precision (a tuning hook, relaxed atomics as
// the kernel-family switch)
static std::atomic<int> g_tile_override[3][2] = {{{0}, {0}}, {{0}, {0}}, {{0}, {0}}};

int dst_set_tile(int kind, int elem_bytes, int pairs) {
  if (kind < 0 || kind > 2 || (elem_bytes != 4 && elem_bytes != 8) || pairs < 0 || (pairs & (pairs - 1)))
    return ST_INVALID;
  g_tile_override[kind][elem_bytes == 8].store(pairs, std::memory_order_relaxed);
  return ST_OK;
}

// Default pencil pairs per work-group.  Strided and fused passes: 16 (FP32) / 8 (FP64)
// pairs, i.e. 128 B row segments, within the launch cap and 150 KB of LDS.  Row passes
// read contiguous pencils, so they take the smallest work-group of at least `row_threads`
// threads: several independent groups per compute unit overlap memory and arithmetic.
int dst_fast_tile(int N, int elem_bytes, int kind) {
  const int tps = fast_tps(N, kind);
  if (!tps) return 0;
  const int ppt = N / tps;
  const bool fused = kind == DST_PASS_FUSED;
  const int cap = ppt <= 16 && !fused ? (elem_bytes == 8 ? 512 : 1024) : (elem_bytes == 8 ? 256 : 512);
  const int stride = (N + (N >> 5) + 1) | 1;
  int nseq = elem_bytes == 8 ? 8 : 16;
  if (kind == DST_PASS_ROWS) {
    const int row_threads = 64;
    nseq = 1;
    while (nseq * tps < row_threads) nseq *= 2;
  }
  while (nseq * tps < 64) nseq *= 2;
  while (nseq > 1 && (nseq * tps > cap || (size_t)nseq * stride * 2 * elem_bytes > 150 * 1024)) nseq /= 2;
  if (nseq * tps > cap || (nseq * tps) % 64) return 0;
  return nseq;
}

template <typename T>
int dst_fast_pass(int N, const cx<T>* tw, const T* sn, const T* in, T* out, long long outer,
                  long long inner, long long pitch, const DstScale<T>* fused, int nseq, hipStream_t st,
                  const DstFaces<T>* faces) {
  if (fused && inner == 1) return ST_INVALID;
  if (faces && (faces->mode < 0 || faces->mode > 1 || (faces->mode == 1 && !fused))) return ST_INVALID;
  // per-lane offsets are 32-bit: one slab (rows: one tile) must stay below 2^31 elements
  if ((double)(N - 1) * (double)inner >= 2147483647.0 || (inner == 1 && 256.0 * pitch >= 2147483647.0))
    return ST_UNSUPPORTED;
  const int kind = fused ? DST_PASS_FUSED : (inner == 1 ? DST_PASS_ROWS : DST_PASS_STRIDED);
  // row passes with the default tile: compile-time row kernel (dst_rows.hip)
  if (kind == DST_PASS_ROWS && nseq <= 0 && g_tile_override[kind][sizeof(T) == 8].load(std::memory_order_relaxed) == 0 && dst_get_variant() != 3) {
    const int rc = dst_rows_pass<T>(N, tw, sn, in, out, outer, pitch, st);
    if (rc != ST_UNSUPPORTED) return rc;
  }
  // strided passes (plain, or forward + scaling + face sums) with the default tile:
  // persistent pipelined kernel (dst_pipe.hip)
  if (inner > 1 && nseq <= 0 && g_tile_override[kind][sizeof(T) == 8].load(std::memory_order_relaxed) == 0 && dst_get_variant() != 3) {
    const int rc = dst_pipe_pass<T>(N, tw, sn, in, out, outer, inner, fused, faces, 0, st);
    if (rc != ST_UNSUPPORTED) return rc;
  }
  fast::Args<T> a;
  a.in = in;
  a.out = out;
  a.tw = tw;
  a.sn = sn;
  a.outer = outer;
  a.inner = inner;
  a.pitch = pitch;
  const int dflt = dst_fast_tile(N, (int)sizeof(T), kind);
  const int ovr = g_tile_override[kind][sizeof(T) == 8].load(std::memory_order_relaxed);
  if (nseq <= 0) nseq = ovr > 0 ? ovr : dflt;
  if (fused && nseq > dflt) nseq = dflt;  // the fused pass has a lower size cap
  if (nseq <= 0 || (nseq & (nseq - 1))) return ST_UNSUPPORTED;
  a.lg_nseq = __builtin_ctz(nseq);
  a.ntile_inner = inner == 1 ? 1 : (inner + 2LL * nseq - 1) / (2LL * nseq);
  if (fused) a.fs = *fused;
  if (faces) a.fc = *faces;
  switch (N) {
    case 32: return fast::launch<T, 32>(a, kind, nseq, st);
    case 64: return fast::launch<T, 64>(a, kind, nseq, st);
    case 96: return fast::launch<T, 96>(a, kind, nseq, st);
    case 128: return fast::launch<T, 128>(a, kind, nseq, st);
    case 192: return fast::launch<T, 192>(a, kind, nseq, st);
    case 256: return fast::launch<T, 256>(a, kind, nseq, st);
    case 384: return fast::launch<T, 384>(a, kind, nseq, st);
    case 512: return fast::launch<T, 512>(a, kind, nseq, st);
    case 768: return fast::launch<T, 768>(a, kind, nseq, st);
    case 1024: return fast::launch<T, 1024>(a, kind, nseq, st);
    case 2048: return fast::launch<T, 2048>(a, kind, nseq, st);
    case 4096: return fast::launch<T, 4096>(a, kind, nseq, st);
    default: return ST_UNSUPPORTED;
  }
}

template int dst_fast_pass<float>(int, const cx<float>*, const float*, const float*, float*, long long,
                                  long long, long long, const DstScale<float>*, int, hipStream_t,
                                  const DstFaces<float>*);
template int dst_fast_pass<double>(int, const cx<double>*, const double*, const double*, double*,
                                   long long, long long, long long, const DstScale<double>*, int, hipStream_t,
                                   const DstFaces<double>*);

}  // namespace ahoc
