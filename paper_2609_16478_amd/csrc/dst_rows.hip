// DST-I pass over contiguous pencils (rows of the fastest axis), gfx950.
//
// The transform is the one of the other pass kernels (two real rows packed in one complex
// FFT, symmetric pre-weighting, split + prefix sum).  This kernel is specialised for the
// row layout: NSEQ row pairs of TPS lanes each per work-group (at least one wavefront),
// all index arithmetic compile-time except the work-group's base row, the rows addressed
// through a uniform base and 32-bit per-lane offsets, and the LDS positions through one
// padded base per direction plus immediate offsets.  Many small work-groups share a compute
// unit, so the load, transform and store phases of different groups overlap.
#include "dst_device.h"

#include <mutex>

namespace ahoc {

namespace fast {

namespace {

template <int N> using RPlan = PlanOf<N, N == 512 || N == 1024>;

// Row loads and stores: non-temporal in FP32 when the array is larger than the caches
// (measured at N = 1024 over the 1023^2 rows: 1.69 -> 1.64 ms), plain otherwise (FP64 at
// N = 1024: 3.65 -> 3.88 ms with non-temporal accesses; small arrays are re-read from the
// caches by the next pass)
template <typename T, bool NT> __device__ __forceinline__ T ldr(const SBase& b, unsigned off) {
  if constexpr (NT) return b.ld_nt<T>(off);
  else return b.ld<T>(off);
}
template <typename T, bool NT> __device__ __forceinline__ void str_(const SBase& b, unsigned off, T v) {
  if constexpr (NT) b.st_nt<T>(off, v);
  else b.st<T>(off, v);
}
template <int N> constexpr int rows_nseq() {
  constexpr int TPS = N / RPlan<N>::PPT;
  return TPS >= 64 ? 1 : 64 / TPS;
}

// LIFT: the input rows are a source plus the face layers of the V-solve's lift, added while
// loading (the lift pass is not run): row r = (j - 1) + (k - 1) n_y' (3-D) or
// (j - 1) + b n_y' (2-D, instance b) gets Lx[side] at its first and last position, and the
// whole row of Ly[side] (Lz[side]) when it lies next to a y (z) face.  Layouts of face_lift.
// ADD: out_row = S in_row + add_row (add with the layout of out), the addend fetched after the
// transform at the store positions.
template <typename T, int N, bool NT, bool LIFT = false, bool ADD = false>
__global__ void __launch_bounds__(rows_nseq<N>()*(N / RPlan<N>::PPT)) k_dst_rows(const T* __restrict__ in,
                                                                                T* __restrict__ out,
                                                                                const cx<T>* __restrict__ tw,
                                                                                const T* __restrict__ sn,
                                                                                long long nrows, long long pitch,
                                                                                RowLift<T> lf = RowLift<T>{},
                                                                                const T* __restrict__ addv = nullptr) {
  extern __shared__ __align__(16) unsigned char smem[];
  using PL = RPlan<N>;
  constexpr int PPT = PL::PPT;
  constexpr int TPS = N / PPT;
  constexpr int NSEQ = rows_nseq<N>();
  constexpr int L = N - 1;
  constexpr int HN = N / 2;
  constexpr int U = PPT / 2;
  constexpr int LDQ = seq_stride<N>();
  constexpr int NTOT = 2 * (TPS / 64 > 0 ? TPS / 64 : 1);
  constexpr bool LIN = TPS % 32 == 0;
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem);
  const int q = threadIdx.x / TPS;  // pair of this thread
  const int t = threadIdx.x - q * TPS;
  cx<T>* seq = lds + q * LDQ;
  cx<T>* tot = lds + NSEQ * LDQ + q * NTOT;
  const long long r0 = (long long)blockIdx.x * (2 * NSEQ);  // first row of the work-group
  const long long ra = r0 + 2 * q;
  const bool oka = ra < nrows, okb = ra + 1 < nrows;
  // rows of the work-group from a uniform base; lane offsets (bytes) stay below 2^32
  const SBase src(in + r0 * pitch);
  const unsigned oa = (unsigned)((2 * q) * pitch * (long long)sizeof(T));
  const unsigned ob = oa + (unsigned)(pitch * (long long)sizeof(T));

  // ---- load + pre-weighting w_m = s_m (z_m + z_{N-m}) + (z_m - z_{N-m}) / 2
  {
    cx<T>* lo = seq + pad(1 + t);
    cx<T>* hi = seq + pad(N - 1 - t);
    T xa[U], xb[U], ya[U], yb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int m = 1 + t + u * TPS;
      const unsigned e1 = (unsigned)((m - 1) * (int)sizeof(T)), e2 = (unsigned)((N - m - 1) * (int)sizeof(T));
      xa[u] = oka ? ldr<T, NT>(src, oa + e1) : T(0);
      xb[u] = okb ? ldr<T, NT>(src, ob + e1) : T(0);
      const bool mid = u == U - 1 && m == HN;
      ya[u] = (oka && !mid) ? ldr<T, NT>(src, oa + e2) : T(0);
      yb[u] = (okb && !mid) ? ldr<T, NT>(src, ob + e2) : T(0);
    }
    if constexpr (LIFT) {
      // the lift's face layers of both rows: x faces at positions 1 and N - 1 (thread 0,
      // u = 0: m = 1 and N - m = N - 1), y and z faces on whole rows next to those faces
      auto add_row = [&](long long r, bool ok, T* x, T* y) {
        if (!ok) return;
        const int j = (int)(r % lf.ni1) + 1;
        const int k = lf.dim == 3 ? (int)(r / lf.ni1) + 1 : 0;
        const long long b = lf.dim == 3 ? 0 : r / lf.ni1;
        if (t == 0) {
          const long long xo = lf.dim == 3 ? (long long)(j - 1) * lf.ni2 + (k - 1) : b * 2 * lf.ni1 + (j - 1);
          x[0] += lf.lx[xo];
          y[0] += lf.lx[xo + lf.xplane];
        }
        const T* rows[2] = {nullptr, nullptr};
        if (lf.dim == 3) {
          if (j == 1) rows[0] = lf.ly + (long long)(k - 1) * lf.px;
          else if (j == lf.ni1) rows[0] = lf.ly + lf.yplane + (long long)(k - 1) * lf.px;
          if (k == 1) rows[1] = lf.lz + (long long)(j - 1) * lf.px;
          else if (k == lf.ni2) rows[1] = lf.lz + lf.zplane + (long long)(j - 1) * lf.px;
        } else {
          if (j == 1) rows[0] = lf.ly + b * 2 * lf.px;
          else if (j == lf.ni1) rows[0] = lf.ly + b * 2 * lf.px + lf.px;
        }
#pragma unroll
        for (int f = 0; f < 2; ++f) {
          if (!rows[f]) continue;
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int m = 1 + t + u * TPS;
            x[u] += rows[f][m - 1];
            if (!(u == U - 1 && m == HN)) y[u] += rows[f][N - m - 1];
          }
        }
      };
      add_row(ra, oka, xa, ya);
      add_row(ra + 1, okb, xb, yb);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int m = 1 + t + u * TPS;
      cx<T>* plo = LIN ? lo + poff(u * TPS) : seq + pad(m);
      cx<T>* phi = LIN ? hi - poff(u * TPS) : seq + pad(N - m);
      if (u == U - 1 && m == HN) {  // the middle position pairs with itself: 2 z
        cx<T> o;
        o.x = T(2) * xa[u];
        o.y = T(2) * xb[u];
        *plo = o;
      } else {
        const T w = sn[m];
        const T sx = w * (xa[u] + ya[u]), sy = w * (xb[u] + yb[u]);
        const T dx = T(0.5) * (xa[u] - ya[u]), dy = T(0.5) * (xb[u] - yb[u]);
        cx<T> o1, o2;
        o1.x = sx + dx;
        o1.y = sy + dy;
        o2.x = sx - dx;
        o2.y = sy - dy;
        *plo = o1;
        *phi = o2;
      }
    }
    if (t == 0) {
      cx<T> z;
      z.x = T(0);
      z.y = T(0);
      seq[0] = z;
    }
  }
  __syncthreads();

  cx<T> A, B;
  A.x = A.y = T(1);
  B.x = B.y = T(0);
  fft<T, N, PL>(seq, t, tw);
  post<T, N, PL, false>(seq, tot, t, A, B, nullptr, T(0));

  // ---- ADD: the addend at the store positions
  [[maybe_unused]] T aa[PPT], ab[PPT];
  if constexpr (ADD) {
    const SBase asrc(addv + r0 * pitch);
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int m = 1 + t + k * TPS;
      const bool in_n = k < PPT - 1 || m < N;
      const unsigned e = (unsigned)((m - 1) * (int)sizeof(T));
      aa[k] = (oka && in_n) ? ldr<T, NT>(asrc, oa + e) : T(0);
      ab[k] = (okb && in_n) ? ldr<T, NT>(asrc, ob + e) : T(0);
    }
  }

  // ---- store positions m = 1 + t + k TPS
  const SBase dst(out + r0 * pitch);
  const cx<T>* lo = seq + pad(1 + t);
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int m = 1 + t + k * TPS;
    if (k < PPT - 1 || m < N) {
      cx<T> v = LIN ? lo[poff(k * TPS)] : seq[pad(m)];
      if constexpr (ADD) {
        v.x += aa[k];
        v.y += ab[k];
      }
      const unsigned e = (unsigned)((m - 1) * (int)sizeof(T));
      if (oka) str_<T, NT>(dst, oa + e, v.x);
      if (okb) str_<T, NT>(dst, ob + e, v.y);
    }
  }
}

// Two DST-I transforms of each row with a pointwise product between them,
//   out_row = S (c_row .* (S in_row)),
// c a nodal array: row r = (j - 1) + (p - kofs) ni1 of the interior (j = 1..ni1, plane or
// instance p) reads c[(p nn1 + j) nn0 + i] at position i = 1..N-1.  The x pass of the Schur
// matvec: the V-solve's last inverse transform, V / alpha, and the U-solve's first forward
// transform in one read and one write of the volume.  The multiplier rows are fetched after
// the first transform; between the transforms every position stays with the thread that
// the store mapping gives it, then the pre-weighting of the second transform reads the
// mirrored positions from LDS.
template <typename T, int N, bool NT>
__global__ void __launch_bounds__(rows_nseq<N>()*(N / RPlan<N>::PPT)) k_dst_rows_mul(
    const T* __restrict__ in, T* __restrict__ out, const cx<T>* __restrict__ tw, const T* __restrict__ sn,
    long long nrows, long long pitch, const T* __restrict__ c, int ni1, int kofs, int nn0, int nn1) {
  extern __shared__ __align__(16) unsigned char smem[];
  using PL = RPlan<N>;
  constexpr int PPT = PL::PPT;
  constexpr int TPS = N / PPT;
  constexpr int NSEQ = rows_nseq<N>();
  constexpr int HN = N / 2;
  constexpr int U = PPT / 2;
  constexpr int LDQ = seq_stride<N>();
  constexpr int NTOT = 2 * (TPS / 64 > 0 ? TPS / 64 : 1);
  constexpr bool LIN = TPS % 32 == 0;
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem);
  const int q = threadIdx.x / TPS;
  const int t = threadIdx.x - q * TPS;
  cx<T>* seq = lds + q * LDQ;
  cx<T>* tot = lds + NSEQ * LDQ + q * NTOT;
  const long long r0 = (long long)blockIdx.x * (2 * NSEQ);
  const long long ra = r0 + 2 * q;
  const bool oka = ra < nrows, okb = ra + 1 < nrows;
  const SBase src(in + r0 * pitch);
  const unsigned oa = (unsigned)((2 * q) * pitch * (long long)sizeof(T));
  const unsigned ob = oa + (unsigned)(pitch * (long long)sizeof(T));

  // ---- load + pre-weighting (as k_dst_rows)
  {
    cx<T>* lo = seq + pad(1 + t);
    cx<T>* hi = seq + pad(N - 1 - t);
    T xa[U], xb[U], ya[U], yb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int m = 1 + t + u * TPS;
      const unsigned e1 = (unsigned)((m - 1) * (int)sizeof(T)), e2 = (unsigned)((N - m - 1) * (int)sizeof(T));
      xa[u] = oka ? ldr<T, NT>(src, oa + e1) : T(0);
      xb[u] = okb ? ldr<T, NT>(src, ob + e1) : T(0);
      const bool mid = u == U - 1 && m == HN;
      ya[u] = (oka && !mid) ? ldr<T, NT>(src, oa + e2) : T(0);
      yb[u] = (okb && !mid) ? ldr<T, NT>(src, ob + e2) : T(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int m = 1 + t + u * TPS;
      cx<T>* plo = LIN ? lo + poff(u * TPS) : seq + pad(m);
      cx<T>* phi = LIN ? hi - poff(u * TPS) : seq + pad(N - m);
      if (u == U - 1 && m == HN) {
        cx<T> o;
        o.x = T(2) * xa[u];
        o.y = T(2) * xb[u];
        *plo = o;
      } else {
        const T w = sn[m];
        const T sx = w * (xa[u] + ya[u]), sy = w * (xb[u] + yb[u]);
        const T dx = T(0.5) * (xa[u] - ya[u]), dy = T(0.5) * (xb[u] - yb[u]);
        cx<T> o1, o2;
        o1.x = sx + dx;
        o1.y = sy + dy;
        o2.x = sx - dx;
        o2.y = sy - dy;
        *plo = o1;
        *phi = o2;
      }
    }
    if (t == 0) {
      cx<T> z;
      z.x = T(0);
      z.y = T(0);
      seq[0] = z;
    }
  }
  __syncthreads();

  cx<T> A, B;
  A.x = A.y = T(1);
  B.x = B.y = T(0);
  fft<T, N, PL>(seq, t, tw);
  post<T, N, PL, false>(seq, tot, t, A, B, nullptr, T(0));

  // ---- multiplier rows at the store positions m = 1 + t + k TPS (fetched here, not
  // before the first transform: held across it they cost occupancy)
  T ma[PPT], mb[PPT];
  {
    const T* rowa = c;
    const T* rowb = c;
    if (oka) {
      const long long p = ra / ni1;
      rowa = c + ((p + kofs) * nn1 + (ra - p * ni1 + 1)) * (long long)nn0;
    }
    if (okb) {
      const long long p = (ra + 1) / ni1;
      rowb = c + ((p + kofs) * nn1 + (ra + 1 - p * ni1 + 1)) * (long long)nn0;
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int m = 1 + t + k * TPS;
      const bool in_n = k < PPT - 1 || m < N;
      ma[k] = (oka && in_n) ? rowa[m] : T(0);
      mb[k] = (okb && in_n) ? rowb[m] : T(0);
    }
  }

  // ---- pointwise product at the thread's own positions, then the second transform
  {
    cx<T>* lo = seq + pad(1 + t);
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int m = 1 + t + k * TPS;
      if (k < PPT - 1 || m < N) {
        cx<T>* pv = LIN ? lo + poff(k * TPS) : seq + pad(m);
        cx<T> v = *pv;
        v.x *= ma[k];
        v.y *= mb[k];
        *pv = v;
      }
    }
  }
  pair_sync<TPS>();
  pre_lds<T, N, PL>(seq, t, sn);
  fft<T, N, PL>(seq, t, tw);
  post<T, N, PL, false>(seq, tot, t, A, B, nullptr, T(0));

  const SBase dst(out + r0 * pitch);
  const cx<T>* lo = seq + pad(1 + t);
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int m = 1 + t + k * TPS;
    if (k < PPT - 1 || m < N) {
      const cx<T> v = LIN ? lo[poff(k * TPS)] : seq[pad(m)];
      const unsigned e = (unsigned)((m - 1) * (int)sizeof(T));
      if (oka) str_<T, NT>(dst, oa + e, v.x);
      if (okb) str_<T, NT>(dst, ob + e, v.y);
    }
  }
}

template <typename T, int N> int rows_mul_launch(const T* in, T* out, const cx<T>* tw, const T* sn, long long nrows,
                                                 long long pitch, const T* c, int ni1, int kofs, int nn0, int nn1,
                                                 hipStream_t st) {
  constexpr int TPS = N / RPlan<N>::PPT;
  constexpr int NSEQ = rows_nseq<N>();
  constexpr int THREADS = NSEQ * TPS;
  constexpr size_t LDS = (size_t)(NSEQ * seq_stride<N>() + NSEQ * 2 * (TPS / 64 > 0 ? TPS / 64 : 1)) * sizeof(cx<T>);
  if (THREADS % 64 != 0 || THREADS > 1024 || LDS > 64 * 1024) return ST_UNSUPPORTED;
  if ((double)(2 * NSEQ) * (double)pitch * (double)sizeof(T) >= 4294967295.0) return ST_UNSUPPORTED;
  const long long blocks = (nrows + 2 * NSEQ - 1) / (2 * NSEQ);
  if (blocks <= 0) return ST_OK;
  if (blocks > 0x7fffffffLL) return ST_UNSUPPORTED;
  if (sizeof(T) == 4 && (double)nrows * (double)pitch * sizeof(T) >= NT_STORE_MIN_BYTES)
    hipLaunchKernelGGL((k_dst_rows_mul<T, N, true>), dim3((unsigned)blocks), dim3(THREADS), LDS, st, in, out, tw, sn,
                       nrows, pitch, c, ni1, kofs, nn0, nn1);
  else
    hipLaunchKernelGGL((k_dst_rows_mul<T, N, false>), dim3((unsigned)blocks), dim3(THREADS), LDS, st, in, out, tw,
                       sn, nrows, pitch, c, ni1, kofs, nn0, nn1);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

template <typename T, int N> int rows_lift_launch(const T* in, T* out, const cx<T>* tw, const T* sn, long long nrows,
                                                  long long pitch, const RowLift<T>& lf, hipStream_t st) {
  constexpr int TPS = N / RPlan<N>::PPT;
  constexpr int NSEQ = rows_nseq<N>();
  constexpr int THREADS = NSEQ * TPS;
  constexpr size_t LDS = (size_t)(NSEQ * seq_stride<N>() + NSEQ * 2 * (TPS / 64 > 0 ? TPS / 64 : 1)) * sizeof(cx<T>);
  if (THREADS % 64 != 0 || THREADS > 1024 || LDS > 64 * 1024) return ST_UNSUPPORTED;
  if ((double)(2 * NSEQ) * (double)pitch * (double)sizeof(T) >= 4294967295.0) return ST_UNSUPPORTED;
  const long long blocks = (nrows + 2 * NSEQ - 1) / (2 * NSEQ);
  if (blocks <= 0) return ST_OK;
  if (blocks > 0x7fffffffLL) return ST_UNSUPPORTED;
  if (sizeof(T) == 4 && (double)nrows * (double)pitch * sizeof(T) >= NT_STORE_MIN_BYTES)
    hipLaunchKernelGGL((k_dst_rows<T, N, true, true>), dim3((unsigned)blocks), dim3(THREADS), LDS, st, in, out, tw,
                       sn, nrows, pitch, lf);
  else
    hipLaunchKernelGGL((k_dst_rows<T, N, false, true>), dim3((unsigned)blocks), dim3(THREADS), LDS, st, in, out,
                       tw, sn, nrows, pitch, lf);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

template <typename T, int N> int rows_add_launch(const T* in, T* out, const cx<T>* tw, const T* sn, long long nrows,
                                                 long long pitch, const T* addv, hipStream_t st) {
  constexpr int TPS = N / RPlan<N>::PPT;
  constexpr int NSEQ = rows_nseq<N>();
  constexpr int THREADS = NSEQ * TPS;
  constexpr size_t LDS = (size_t)(NSEQ * seq_stride<N>() + NSEQ * 2 * (TPS / 64 > 0 ? TPS / 64 : 1)) * sizeof(cx<T>);
  if (THREADS % 64 != 0 || THREADS > 1024 || LDS > 64 * 1024) return ST_UNSUPPORTED;
  if ((double)(2 * NSEQ) * (double)pitch * (double)sizeof(T) >= 4294967295.0) return ST_UNSUPPORTED;
  const long long blocks = (nrows + 2 * NSEQ - 1) / (2 * NSEQ);
  if (blocks <= 0) return ST_OK;
  if (blocks > 0x7fffffffLL) return ST_UNSUPPORTED;
  if (sizeof(T) == 4 && (double)nrows * (double)pitch * sizeof(T) >= NT_STORE_MIN_BYTES)
    hipLaunchKernelGGL((k_dst_rows<T, N, true, false, true>), dim3((unsigned)blocks), dim3(THREADS), LDS, st, in, out,
                       tw, sn, nrows, pitch, RowLift<T>{}, addv);
  else
    hipLaunchKernelGGL((k_dst_rows<T, N, false, false, true>), dim3((unsigned)blocks), dim3(THREADS), LDS, st, in,
                       out, tw, sn, nrows, pitch, RowLift<T>{}, addv);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

template <typename T, int N> int rows_launch(const T* in, T* out, const cx<T>* tw, const T* sn, long long nrows,
                                             long long pitch, hipStream_t st) {
  constexpr int TPS = N / RPlan<N>::PPT;
  constexpr int NSEQ = rows_nseq<N>();
  constexpr int THREADS = NSEQ * TPS;
  constexpr size_t LDS = (size_t)(NSEQ * seq_stride<N>() + NSEQ * 2 * (TPS / 64 > 0 ? TPS / 64 : 1)) * sizeof(cx<T>);
  if (THREADS % 64 != 0 || THREADS > 1024 || LDS > 64 * 1024) return ST_UNSUPPORTED;
  // per-lane byte offsets within a work-group's rows
  if ((double)(2 * NSEQ) * (double)pitch * (double)sizeof(T) >= 4294967295.0) return ST_UNSUPPORTED;
  const long long blocks = (nrows + 2 * NSEQ - 1) / (2 * NSEQ);
  if (blocks <= 0) return ST_OK;
  if (blocks > 0x7fffffffLL) return ST_UNSUPPORTED;
  if (sizeof(T) == 4 && (double)nrows * (double)pitch * sizeof(T) >= NT_STORE_MIN_BYTES)
    hipLaunchKernelGGL((k_dst_rows<T, N, true>), dim3((unsigned)blocks), dim3(THREADS), LDS, st, in, out, tw, sn,
                       nrows, pitch);
  else
    hipLaunchKernelGGL((k_dst_rows<T, N, false>), dim3((unsigned)blocks), dim3(THREADS), LDS, st, in, out, tw, sn,
                       nrows, pitch);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

}  // namespace

}  // namespace fast

template <typename T>
int dst_rows_pass(int N, const cx<T>* tw, const T* sn, const T* in, T* out, long long nrows, long long pitch,
                  hipStream_t st) {
  if (pitch < N - 1) return ST_INVALID;
  switch (N) {
    case 32: return fast::rows_launch<T, 32>(in, out, tw, sn, nrows, pitch, st);
    case 64: return fast::rows_launch<T, 64>(in, out, tw, sn, nrows, pitch, st);
    case 96: return fast::rows_launch<T, 96>(in, out, tw, sn, nrows, pitch, st);
    case 128: return fast::rows_launch<T, 128>(in, out, tw, sn, nrows, pitch, st);
    case 192: return fast::rows_launch<T, 192>(in, out, tw, sn, nrows, pitch, st);
    case 256: return fast::rows_launch<T, 256>(in, out, tw, sn, nrows, pitch, st);
    case 384: return fast::rows_launch<T, 384>(in, out, tw, sn, nrows, pitch, st);
    case 512: return fast::rows_launch<T, 512>(in, out, tw, sn, nrows, pitch, st);
    case 768: return fast::rows_launch<T, 768>(in, out, tw, sn, nrows, pitch, st);
    case 1024: return fast::rows_launch<T, 1024>(in, out, tw, sn, nrows, pitch, st);
    case 2048: return fast::rows_launch<T, 2048>(in, out, tw, sn, nrows, pitch, st);
    case 4096: return fast::rows_launch<T, 4096>(in, out, tw, sn, nrows, pitch, st);
    default: return ST_UNSUPPORTED;
  }
}

namespace fast {
namespace {
template <typename T, int N> bool rows_lift_ok(long long nrows, long long pitch) {
  constexpr int TPS = N / RPlan<N>::PPT;
  constexpr int NSEQ = rows_nseq<N>();
  constexpr int THREADS = NSEQ * TPS;
  constexpr size_t LDS = (size_t)(NSEQ * seq_stride<N>() + NSEQ * 2 * (TPS / 64 > 0 ? TPS / 64 : 1)) * sizeof(cx<T>);
  return THREADS % 64 == 0 && THREADS <= 1024 && LDS <= 64 * 1024 &&
         (double)(2 * NSEQ) * (double)pitch * (double)sizeof(T) < 4294967295.0 &&
         (nrows + 2 * NSEQ - 1) / (2 * NSEQ) <= 0x7fffffffLL;
}
}  // namespace
}  // namespace fast

template <typename T> bool dst_rows_lift_supported(int N, long long nrows, long long pitch) {
  if (pitch < N - 1) return false;
  switch (N) {
    case 32: return fast::rows_lift_ok<T, 32>(nrows, pitch);
    case 64: return fast::rows_lift_ok<T, 64>(nrows, pitch);
    case 96: return fast::rows_lift_ok<T, 96>(nrows, pitch);
    case 128: return fast::rows_lift_ok<T, 128>(nrows, pitch);
    case 192: return fast::rows_lift_ok<T, 192>(nrows, pitch);
    case 256: return fast::rows_lift_ok<T, 256>(nrows, pitch);
    case 384: return fast::rows_lift_ok<T, 384>(nrows, pitch);
    case 512: return fast::rows_lift_ok<T, 512>(nrows, pitch);
    case 768: return fast::rows_lift_ok<T, 768>(nrows, pitch);
    case 1024: return fast::rows_lift_ok<T, 1024>(nrows, pitch);
    case 2048: return fast::rows_lift_ok<T, 2048>(nrows, pitch);
    case 4096: return fast::rows_lift_ok<T, 4096>(nrows, pitch);
    default: return false;
  }
}
template bool dst_rows_lift_supported<float>(int, long long, long long);
template bool dst_rows_lift_supported<double>(int, long long, long long);

template <typename T>
int dst_rows_lift_pass(int N, const cx<T>* tw, const T* sn, const T* in, T* out, long long nrows, long long pitch,
                       const RowLift<T>& lf, hipStream_t st) {
  if (pitch < N - 1 || lf.ni1 <= 0 || (lf.dim != 2 && lf.dim != 3)) return ST_INVALID;
  switch (N) {
    case 32: return fast::rows_lift_launch<T, 32>(in, out, tw, sn, nrows, pitch, lf, st);
    case 64: return fast::rows_lift_launch<T, 64>(in, out, tw, sn, nrows, pitch, lf, st);
    case 96: return fast::rows_lift_launch<T, 96>(in, out, tw, sn, nrows, pitch, lf, st);
    case 128: return fast::rows_lift_launch<T, 128>(in, out, tw, sn, nrows, pitch, lf, st);
    case 192: return fast::rows_lift_launch<T, 192>(in, out, tw, sn, nrows, pitch, lf, st);
    case 256: return fast::rows_lift_launch<T, 256>(in, out, tw, sn, nrows, pitch, lf, st);
    case 384: return fast::rows_lift_launch<T, 384>(in, out, tw, sn, nrows, pitch, lf, st);
    case 512: return fast::rows_lift_launch<T, 512>(in, out, tw, sn, nrows, pitch, lf, st);
    case 768: return fast::rows_lift_launch<T, 768>(in, out, tw, sn, nrows, pitch, lf, st);
    case 1024: return fast::rows_lift_launch<T, 1024>(in, out, tw, sn, nrows, pitch, lf, st);
    case 2048: return fast::rows_lift_launch<T, 2048>(in, out, tw, sn, nrows, pitch, lf, st);
    case 4096: return fast::rows_lift_launch<T, 4096>(in, out, tw, sn, nrows, pitch, lf, st);
    default: return ST_UNSUPPORTED;
  }
}
template int dst_rows_lift_pass<float>(int, const cx<float>*, const float*, const float*, float*, long long, long long,
                                       const RowLift<float>&, hipStream_t);
template int dst_rows_lift_pass<double>(int, const cx<double>*, const double*, const double*, double*, long long,
                                        long long, const RowLift<double>&, hipStream_t);

template <typename T>
int dst_rows_add_pass(int N, const cx<T>* tw, const T* sn, const T* in, T* out, const T* addv, long long nrows,
                      long long pitch, hipStream_t st) {
  if (pitch < N - 1 || !addv) return ST_INVALID;
  switch (N) {
#define AHOC_RADD(NN) \
  case NN: return fast::rows_add_launch<T, NN>(in, out, tw, sn, nrows, pitch, addv, st);
    AHOC_RADD(32) AHOC_RADD(64) AHOC_RADD(96) AHOC_RADD(128) AHOC_RADD(192) AHOC_RADD(256)
    AHOC_RADD(384) AHOC_RADD(512) AHOC_RADD(768) AHOC_RADD(1024) AHOC_RADD(2048) AHOC_RADD(4096)
#undef AHOC_RADD
    default: return ST_UNSUPPORTED;
  }
}
template int dst_rows_add_pass<float>(int, const cx<float>*, const float*, const float*, float*, const float*,
                                      long long, long long, hipStream_t);
template int dst_rows_add_pass<double>(int, const cx<double>*, const double*, const double*, double*, const double*,
                                       long long, long long, hipStream_t);

template <typename T>
int dst_rows_mul_pass(int N, const cx<T>* tw, const T* sn, const T* in, T* out, long long nrows, long long pitch,
                      const T* c, int ni1, int kofs, int nn0, int nn1, hipStream_t st) {
  if (pitch < N - 1 || ni1 <= 0 || nn0 < N + 1) return ST_INVALID;
  switch (N) {
    case 32: return fast::rows_mul_launch<T, 32>(in, out, tw, sn, nrows, pitch, c, ni1, kofs, nn0, nn1, st);
    case 64: return fast::rows_mul_launch<T, 64>(in, out, tw, sn, nrows, pitch, c, ni1, kofs, nn0, nn1, st);
    case 96: return fast::rows_mul_launch<T, 96>(in, out, tw, sn, nrows, pitch, c, ni1, kofs, nn0, nn1, st);
    case 128: return fast::rows_mul_launch<T, 128>(in, out, tw, sn, nrows, pitch, c, ni1, kofs, nn0, nn1, st);
    case 192: return fast::rows_mul_launch<T, 192>(in, out, tw, sn, nrows, pitch, c, ni1, kofs, nn0, nn1, st);
    case 256: return fast::rows_mul_launch<T, 256>(in, out, tw, sn, nrows, pitch, c, ni1, kofs, nn0, nn1, st);
    case 384: return fast::rows_mul_launch<T, 384>(in, out, tw, sn, nrows, pitch, c, ni1, kofs, nn0, nn1, st);
    case 512: return fast::rows_mul_launch<T, 512>(in, out, tw, sn, nrows, pitch, c, ni1, kofs, nn0, nn1, st);
    case 768: return fast::rows_mul_launch<T, 768>(in, out, tw, sn, nrows, pitch, c, ni1, kofs, nn0, nn1, st);
    case 1024: return fast::rows_mul_launch<T, 1024>(in, out, tw, sn, nrows, pitch, c, ni1, kofs, nn0, nn1, st);
    case 2048: return fast::rows_mul_launch<T, 2048>(in, out, tw, sn, nrows, pitch, c, ni1, kofs, nn0, nn1, st);
    case 4096: return fast::rows_mul_launch<T, 4096>(in, out, tw, sn, nrows, pitch, c, ni1, kofs, nn0, nn1, st);
    default: return ST_UNSUPPORTED;
  }
}

template int dst_rows_mul_pass<float>(int, const cx<float>*, const float*, const float*, float*, long long, long long,
                                      const float*, int, int, int, int, hipStream_t);
template int dst_rows_mul_pass<double>(int, const cx<double>*, const double*, const double*, double*, long long,
                                       long long, const double*, int, int, int, int, hipStream_t);

template int dst_rows_pass<float>(int, const cx<float>*, const float*, const float*, float*, long long, long long,
                                  hipStream_t);
template int dst_rows_pass<double>(int, const cx<double>*, const double*, const double*, double*, long long,
                                   long long, hipStream_t);

}  // namespace ahoc
