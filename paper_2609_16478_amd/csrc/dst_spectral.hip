// Spectral entry and exit of the Schur matrix-vector product (gfx950).
//
// Both DST-I solves of Lemma 1 touch the boundary only through thin data:
//
//  * V-solve.  The homogeneous right-hand side L_h^bnd[Q] is non-zero only on the
//    interior layers next to the faces, and on each such layer it is a tangential
//    stencil of one face's Q.  Its 3-D sine spectrum is therefore a sum of separable
//    terms, one per face: (2-D spectrum of the face layer) x (sine of the layer's
//    position along the normal), sin(pi k / N) for the low face and
//    sin(pi k (N-1) / N) = (-1)^(k+1) sin(pi k / N) for the high face.  k_dst_gen
//    builds each pencil of that spectrum along the slowest axis from the small face
//    spectra, divides by the eigenvalues and applies the inverse transform along that
//    axis: the lift kernel and the two forward passes of the V-solve disappear, and
//    the first remaining pass reads (almost) nothing from HBM.
//
//  * U-solve.  The boundary gather needs U only through the one-sided combination
//    6 U_1 - 3/2 U_2 + 2/9 U_3 next to each face, which is a weighted sum over the
//    sine modes along the face normal.  The slowest-axis pass therefore stops after
//    the forward transform and the eigen scaling (forming the sums along its own axis
//    on the way), and k_face_reduce streams the scaled spectrum once to form the sums
//    along the other two axes: row dots along the fastest axis and weighted column sums
//    along the middle axis of each plane.  No inverse transform of the volume is run,
//    and 2-D inverse transforms of the small face arrays finish the combination.
//
// Column decode of a slab of `inner` pencils: col = ia + na * ib (na = row pitch,
// ia < nva valid); in 2-D ib = 0.
#include "dst_device.h"

#include <mutex>

namespace ahoc {
namespace fast {

template <typename T> struct GenArgs {
  T* out;
  const cx<T>* tw;
  const T* sn;
  long long inner, ntile_inner;
  int lg_nseq;
  DstScale<T> fs;
  DstGen<T> g;
};

// eigenvalue coefficients of column col: lambda(m) = A + B s_this(m)
template <typename T>
__device__ __forceinline__ bool col_coef(const DstScale<T>& fs, long long inner, long long col, int& ia, int& ib,
                                         T& A, T& B) {
  ib = (int)(col / fs.na);
  ia = (int)(col - (long long)ib * fs.na);
  if (col >= inner || ia >= fs.nva) {
    A = 1;
    B = 0;
    return false;
  }
  const T sa = fs.s_a[ia];
  const T sb = fs.s_b ? fs.s_b[ib] : T(0);
  A = sa + sb + fs.c_ab * sa * sb + (fs.a0 + fs.ka * sa + fs.kb * sb);  // + v-equation shift
  B = T(1) + fs.c_ta * sa + fs.c_tb * sb + fs.kt;
  return true;
}

template <typename T, int N>
__global__ void __launch_bounds__((cap<T, N, true, false>())) k_dst_gen(GenArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  using PL = Plan<N>;
  constexpr int PPT = PL::PPT;
  constexpr int TPS = N / PPT;
  constexpr int L = N - 1;
  constexpr int LDQ = seq_stride<N>();
  constexpr int NTOT = 2 * (TPS / 64 > 0 ? TPS / 64 : 1);
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem);
  const int nseq = blockDim.x / TPS;
  const int lgq = a.lg_nseq;
  const int P = 2 * nseq;
  const long long o = blockIdx.x / a.ntile_inner;  // slab (instance of a batch)
  const long long c0 = (blockIdx.x - o * a.ntile_inner) * (long long)P;
  const long long left = a.inner - c0;
  const int ncols = left < P ? (int)left : P;

  // ---- generate the scaled spectrum: item (pair q, position m), q fastest, so that a
  // thread keeps one pencil pair and the lanes of a wavefront read consecutive columns
  {
    DstGen<T> g = a.g;
    g.lp += o * g.pslab;
    g.la += o * g.aslab;
    if (g.lb) g.lb += o * g.bslab;
    const int q = threadIdx.x & (nseq - 1);
    const long long ca = c0 + 2 * q, cb = ca + 1;
    int iaa, iba, iab, ibb;
    T Aa, Ba, Ab, Bb;
    const bool va = col_coef(a.fs, a.inner, ca, iaa, iba, Aa, Ba);
    const bool vb = col_coef(a.fs, a.inner, cb, iab, ibb, Ab, Bb);
    const T pla = va ? g.lp[ca] : T(0), pha = va ? g.lp[g.pplane + ca] : T(0);
    const T plb = vb ? g.lp[cb] : T(0), phb = vb ? g.lp[g.pplane + cb] : T(0);
    const T wla = va ? g.wa[iaa] : T(0), wha = va ? g.wa[g.nwa + iaa] : T(0);
    const T wlb = vb ? g.wa[iab] : T(0), whb = vb ? g.wa[g.nwa + iab] : T(0);
    const T* ra = g.la + (long long)(va ? iba : 0) * g.arow;
    const T* rb = g.la + (long long)(vb ? ibb : 0) * g.arow;
    T bla = 0, bha = 0, blb = 0, bhb = 0;
    const T *sa = g.la, *sb = g.la;
    if (g.lb) {
      bla = va ? g.wb[iba] : T(0);
      bha = va ? g.wb[g.nwb + iba] : T(0);
      blb = vb ? g.wb[ibb] : T(0);
      bhb = vb ? g.wb[g.nwb + ibb] : T(0);
      sa = g.lb + (va ? iaa : 0);
      sb = g.lb + (vb ? iab : 0);
    }
    const T scale = a.fs.scale;
    cx<T>* sq = lds + q * LDQ;
    const int items = nseq * L;
    const bool has_b = g.lb != nullptr;
    constexpr int U = 4;  // items per thread in flight: the face rows come from L2
    for (int i0 = threadIdx.x; i0 < items; i0 += U * (int)blockDim.x) {
      T ga[U], gb[U], st[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int it = i0 + u * (int)blockDim.x;
        const int m = it < items ? 1 + (it >> lgq) : 1;
        const T wpl = g.wp[m - 1], wph = g.wp[L + m - 1];
        const int oa = (m - 1) * g.apitch;
        ga[u] = pla * wpl + pha * wph + ra[oa] * wla + ra[g.aplane + oa] * wha;
        gb[u] = plb * wpl + phb * wph + rb[oa] * wlb + rb[g.aplane + oa] * whb;
        if (has_b) {
          const int ob = (m - 1) * g.bpitch;
          ga[u] += sa[ob] * bla + sa[g.bplane + ob] * bha;
          gb[u] += sb[ob] * blb + sb[g.bplane + ob] * bhb;
        }
        st[u] = a.fs.s_this[m - 1];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int it = i0 + u * (int)blockDim.x;
        if (it < items) {
          const int m = 1 + (it >> lgq);
          cx<T> o;
          o.x = va ? ga[u] * (scale * recip(Aa + Ba * st[u])) : T(0);
          o.y = vb ? gb[u] * (scale * recip(Ab + Bb * st[u])) : T(0);
          sq[pad(m)] = o;
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
  __syncthreads();

  // ---- inverse transform along the pass axis and store
  const int s = threadIdx.x / TPS;
  const int ts = threadIdx.x - s * TPS;
  cx<T>* seq = lds + s * LDQ;
  cx<T>* tot = lds + nseq * LDQ + s * NTOT;
  cx<T> A, B;
  A.x = A.y = T(1);
  B.x = B.y = T(0);
  pre_lds<T, N, PL>(seq, ts, a.sn);
  fft<T, N, PL>(seq, ts, a.tw);
  post<T, N, PL, false>(seq, tot, ts, A, B, nullptr, T(0));
  __syncthreads();  // the store reads other pairs' sequences
  store_tile<T, N>(lds, a.out + o * (long long)L * a.inner + c0, false, nseq, lgq, ncols, (int)a.inner, 1);
}

// Face contractions of a stored scaled spectrum, one work-group per (plane, row chunk):
// row dots with wx through wavefront reductions, and (fy != null, whole planes only)
// column sums with wy accumulated in registers, CPT columns per thread.
template <typename T, int CPT>
__global__ void __launch_bounds__(256) k_face_reduce(const T* __restrict__ W, long long planes, int ny, int nx,
                                                     int px, int rows_per, const T* __restrict__ wx,
                                                     const T* __restrict__ wy, T* __restrict__ fx,
                                                     T* __restrict__ fy, long long fx_side, long long fx_plane,
                                                     long long fx_row) {
  __shared__ T red[2][64][4];
  const int nchunk = (ny + rows_per - 1) / rows_per;
  const long long o = blockIdx.x / nchunk;
  const int r0 = (int)(blockIdx.x - o * nchunk) * rows_per;
  const int r1 = min(ny, r0 + rows_per);
  const T* __restrict__ Wp = W + o * (long long)ny * px;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  T wxl[CPT], wxh[CPT], accl[CPT], acch[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int c = threadIdx.x + 256 * j;
    wxl[j] = c < nx ? wx[c] : T(0);
    wxh[j] = c < nx ? wx[nx + c] : T(0);
    accl[j] = acch[j] = T(0);
  }
  for (int b0 = r0; b0 < r1; b0 += 64) {
    const int rn = min(64, r1 - b0);
#pragma unroll 2
    for (int rr = 0; rr < rn; ++rr) {
      const int ky = b0 + rr;
      const T* __restrict__ row = Wp + (long long)ky * px;
      T v[CPT];
#pragma unroll
      for (int j = 0; j < CPT; ++j) {
        const int c = threadIdx.x + 256 * j;
        v[j] = c < px ? row[c] : T(0);
      }
      T dl = 0, dh = 0;
#pragma unroll
      for (int j = 0; j < CPT; ++j) {
        dl += v[j] * wxl[j];
        dh += v[j] * wxh[j];
      }
      if (fy) {
        const T yl = wy[ky], yh = wy[ny + ky];
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
          accl[j] += v[j] * yl;
          acch[j] += v[j] * yh;
        }
      }
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) {
        dl += __shfl_xor(dl, m, 64);
        dh += __shfl_xor(dh, m, 64);
      }
      if (lane == 0) {
        red[0][rr][wv] = dl;
        red[1][rr][wv] = dh;
      }
    }
    __syncthreads();
    if (threadIdx.x < 2 * rn) {
      const int sd = threadIdx.x >= rn;
      const int rr = threadIdx.x - sd * rn;
      const T t = red[sd][rr][0] + red[sd][rr][1] + red[sd][rr][2] + red[sd][rr][3];
      fx[sd * fx_side + o * fx_plane + (b0 + rr) * fx_row] = t;
    }
    __syncthreads();
  }
  if (fy) {
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const int c = threadIdx.x + 256 * j;
      if (c < px) {
        fy[o * px + c] = accl[j];
        fy[(planes + o) * px + c] = acch[j];
      }
    }
  }
}

template <typename F> void max_lds(F* f) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(f), hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
}

template <typename T, int N>
int gen_launch(const GenArgs<T>& a0, long long outer, hipStream_t st) {
  constexpr int TPS = N / Plan<N>::PPT;
  const int nseq = dst_fast_tile(N, (int)sizeof(T), DST_PASS_FUSED);
  if (nseq <= 0) return ST_UNSUPPORTED;
  GenArgs<T> a = a0;
  a.lg_nseq = __builtin_ctz(nseq);
  const int threads = nseq * TPS;
  if (threads > cap<T, N, true, false>() || threads % 64) return ST_UNSUPPORTED;
  const int ntot = nseq * 2 * (TPS / 64 > 0 ? TPS / 64 : 1);
  const size_t lds = (size_t)(nseq * seq_stride<N>() + ntot) * sizeof(cx<T>);
  if (lds > 160 * 1024) return ST_UNSUPPORTED;
  a.ntile_inner = (a.inner + 2 * nseq - 1) / (2 * nseq);
  const long long blocks = a.ntile_inner * outer;
  if (blocks <= 0) return ST_OK;
  if (blocks > 0x7fffffffLL) return ST_UNSUPPORTED;
  static std::once_flag once;
  std::call_once(once, [] { max_lds(&k_dst_gen<T, N>); });
  hipLaunchKernelGGL((k_dst_gen<T, N>), dim3((unsigned)blocks), dim3(threads), lds, st, a);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

// Face contractions of whole planes (x-face row dots and y-face column sums), one wavefront
// per row: a lane holds CPL = px / 64 columns, so a row's dot needs one wavefront reduction
// for 64 * CPL values; the column sums accumulate per wavefront in registers and are
// combined through LDS once per plane.
template <typename T, int CPL>
__global__ void __launch_bounds__(256) k_face_reduce_w(const T* __restrict__ W, long long planes, int ny, int nx,
                                                       int px, const T* __restrict__ wx, const T* __restrict__ wy,
                                                       T* __restrict__ fx, T* __restrict__ fy, long long fx_side,
                                                       long long fx_plane, long long fx_row) {
  __shared__ T col[4][2][CPL * 64];
  const long long o = blockIdx.x;
  const T* __restrict__ Wp = W + o * (long long)ny * px;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  T wxl[CPL], wxh[CPL], accl[CPL], acch[CPL];
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const int c = lane + 64 * j;
    wxl[j] = c < nx ? wx[c] : T(0);
    wxh[j] = c < nx ? wx[nx + c] : T(0);
    accl[j] = acch[j] = T(0);
  }
#pragma unroll 2
  for (int ky = wv; ky < ny; ky += 4) {
    const T* __restrict__ row = Wp + (long long)ky * px;
    T v[CPL];
#pragma unroll
    for (int j = 0; j < CPL; ++j) v[j] = __builtin_nontemporal_load(row + lane + 64 * j);  // read once
    const T yl = wy[ky], yh = wy[ny + ky];
    T dl = 0, dh = 0;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      dl += v[j] * wxl[j];
      dh += v[j] * wxh[j];
      accl[j] += v[j] * yl;
      acch[j] += v[j] * yh;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      dl += __shfl_xor(dl, m, 64);
      dh += __shfl_xor(dh, m, 64);
    }
    if (lane == 0) {
      fx[o * fx_plane + ky * fx_row] = dl;
      fx[fx_side + o * fx_plane + ky * fx_row] = dh;
    }
  }
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    col[wv][0][lane + 64 * j] = accl[j];
    col[wv][1][lane + 64 * j] = acch[j];
  }
  __syncthreads();
  for (int c = threadIdx.x; c < px; c += 256) {
    fy[o * px + c] = col[0][0][c] + col[1][0][c] + col[2][0][c] + col[3][0][c];
    fy[(planes + o) * px + c] = col[0][1][c] + col[1][1][c] + col[2][1][c] + col[3][1][c];
  }
}

// Row dots alone (no column sums): one wavefront per RPW rows of any plane (row r of the
// planes' stack at W + r px), the RPW x CPL loads of a column chunk issued together, the
// dots reduced with shuffles; no work-group barrier, so every row of a batch of small
// planes is in flight at once.  Columns from nx on are not read.
template <typename T, int CPL, int RPW>
__global__ void __launch_bounds__(256) k_face_rows(const T* __restrict__ W, long long nrows, int ny, int nx, int px,
                                                   const T* __restrict__ wx, T* __restrict__ fx, long long fx_side,
                                                   long long fx_plane, long long fx_row) {
  const int lane = threadIdx.x & 63;
  const long long r0 = ((long long)blockIdx.x * 4 + (threadIdx.x >> 6)) * RPW;
  if (r0 >= nrows) return;  // whole wavefronts only
  T dl[RPW], dh[RPW];
#pragma unroll
  for (int i = 0; i < RPW; ++i) dl[i] = dh[i] = T(0);
  for (int c0 = 0; c0 < nx; c0 += 64 * CPL) {
    T v[RPW][CPL];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const bool okr = r0 + i < nrows;
      const T* __restrict__ row = W + (r0 + i) * (long long)px;
#pragma unroll
      for (int j = 0; j < CPL; ++j) {
        const int c = c0 + lane + 64 * j;
        v[i][j] = (okr && c < nx) ? row[c] : T(0);
      }
    }
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      const int c = c0 + lane + 64 * j;
      const T wl = c < nx ? wx[c] : T(0), wh = c < nx ? wx[nx + c] : T(0);
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
        dl[i] += v[i][j] * wl;
        dh[i] += v[i][j] * wh;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      dl[i] += __shfl_xor(dl[i], m, 64);
      dh[i] += __shfl_xor(dh[i], m, 64);
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const long long r = r0 + i;
      if (r < nrows) {
        const long long o = r / ny, ky = r - o * ny;
        fx[o * fx_plane + ky * fx_row] = dl[i];
        fx[fx_side + o * fx_plane + ky * fx_row] = dh[i];
      }
    }
  }
}

}  // namespace fast

template <typename T>
int dst_gen_pass(const DstTables<T>& tb, T* out, long long outer, long long inner, const DstScale<T>& sc,
                 const DstGen<T>& gen, hipStream_t st) {
  if (!dst_fast_supported(tb.N)) return ST_UNSUPPORTED;
  if ((double)(tb.N - 1) * (double)inner >= 2147483647.0) return ST_UNSUPPORTED;
  if (dst_get_variant() != 3) {  // persistent kernel where its layout conditions hold
    const int rc = dst_gen_pipe_pass<T>(tb, out, outer, inner, sc, gen, st);
    if (rc != ST_UNSUPPORTED) return rc;
  }
  fast::GenArgs<T> a;
  a.out = out;
  a.tw = tb.tw;
  a.sn = tb.sn;
  a.inner = inner;
  a.lg_nseq = 0;
  a.fs = sc;
  a.g = gen;
  switch (tb.N) {
    case 32: return fast::gen_launch<T, 32>(a, outer, st);
    case 64: return fast::gen_launch<T, 64>(a, outer, st);
    case 96: return fast::gen_launch<T, 96>(a, outer, st);
    case 128: return fast::gen_launch<T, 128>(a, outer, st);
    case 192: return fast::gen_launch<T, 192>(a, outer, st);
    case 256: return fast::gen_launch<T, 256>(a, outer, st);
    case 384: return fast::gen_launch<T, 384>(a, outer, st);
    case 512: return fast::gen_launch<T, 512>(a, outer, st);
    case 768: return fast::gen_launch<T, 768>(a, outer, st);
    case 1024: return fast::gen_launch<T, 1024>(a, outer, st);
    case 2048: return fast::gen_launch<T, 2048>(a, outer, st);
    case 4096: return fast::gen_launch<T, 4096>(a, outer, st);
    default: return ST_UNSUPPORTED;
  }
}

template <typename T>
int face_reduce(const T* W, long long planes, int ny, int nx, int px, const T* wx, const T* wy, T* fx, T* fy,
                long long fx_side, long long fx_plane, long long fx_row, hipStream_t st) {
  if (planes <= 0 || ny <= 0) return ST_OK;
  // FP32: one wavefront per row (the FP64 form keeps the 256-lane rows: its 16-column
  // wavefront variant loses occupancy to registers and measured slower)
  if (sizeof(T) == 4 && fy && px % 64 == 0 && px <= 1024 && planes <= 0x7fffffffLL) {
#define AHOC_FRW(C)                                                                                     \
  case C:                                                                                               \
    hipLaunchKernelGGL((fast::k_face_reduce_w<T, C>), dim3((unsigned)planes), dim3(256), 0, st, W, planes, ny, \
                       nx, px, wx, wy, fx, fy, fx_side, fx_plane, fx_row);                              \
    AHOC_HIP_TRY(hipGetLastError());                                                                    \
    return ST_OK
    switch (px / 64) {
      AHOC_FRW(1);
      AHOC_FRW(2);
      AHOC_FRW(3);
      AHOC_FRW(4);
      AHOC_FRW(6);
      AHOC_FRW(8);
      AHOC_FRW(12);
      AHOC_FRW(16);
      default:
        break;
    }
#undef AHOC_FRW
  }
  if (!fy) {
    // row dots alone: one wavefront per 8 / CPL rows (CPL columns per lane and chunk)
    const long long nrows = planes * (long long)ny;
    const int cpl = px <= 64 ? 1 : px <= 128 ? 2 : px <= 256 ? 4 : 8;
    const long long waves = (nrows + 8 / cpl - 1) / (8 / cpl);
    const long long blocks = (waves + 3) / 4;
    if (blocks > 0x7fffffffLL) return ST_UNSUPPORTED;
#define AHOC_FROWS(C)                                                                                     \
  hipLaunchKernelGGL((fast::k_face_rows<T, C, 8 / C>), dim3((unsigned)blocks), dim3(256), 0, st, W, nrows, ny, nx, \
                     px, wx, fx, fx_side, fx_plane, fx_row)
    if (cpl == 1) AHOC_FROWS(1);
    else if (cpl == 2) AHOC_FROWS(2);
    else if (cpl == 4) AHOC_FROWS(4);
    else AHOC_FROWS(8);
#undef AHOC_FROWS
    AHOC_HIP_TRY(hipGetLastError());
    return ST_OK;
  }
  const int cpt = (px + 255) / 256;
  // whole planes when column sums are formed
  const int rows_per = ny;
  const long long nchunk = (ny + rows_per - 1) / rows_per;
  const long long blocks = planes * nchunk;
  if (blocks > 0x7fffffffLL) return ST_UNSUPPORTED;
#define AHOC_FR(C)                                                                                          \
  hipLaunchKernelGGL((fast::k_face_reduce<T, C>), dim3((unsigned)blocks), dim3(256), 0, st, W, planes, ny, nx, \
                     px, rows_per, wx, wy, fx, fy, fx_side, fx_plane, fx_row)
  if (cpt <= 1) AHOC_FR(1);
  else if (cpt <= 2) AHOC_FR(2);
  else if (cpt <= 4) AHOC_FR(4);
  else if (cpt <= 8) AHOC_FR(8);
  else if (cpt <= 16) AHOC_FR(16);
  else return ST_UNSUPPORTED;
#undef AHOC_FR
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

template int dst_gen_pass<float>(const DstTables<float>&, float*, long long, long long, const DstScale<float>&,
                                 const DstGen<float>&, hipStream_t);
template int dst_gen_pass<double>(const DstTables<double>&, double*, long long, long long,
                                  const DstScale<double>&, const DstGen<double>&, hipStream_t);
template int face_reduce<float>(const float*, long long, int, int, int, const float*, const float*, float*,
                                float*, long long, long long, long long, hipStream_t);
template int face_reduce<double>(const double*, long long, int, int, int, const double*, const double*,
                                 double*, double*, long long, long long, long long, hipStream_t);

}  // namespace ahoc
