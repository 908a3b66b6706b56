// Persistent, software-pipelined DST-I pass over strided pencils (gfx950).
//
// The strided passes (pencils along y or z, the fastest axis across pencils) hold a whole
// tile of 2*NSEQ pencils in LDS: at N = 1024 that is ~135 KB, so one work-group fills a
// compute unit and, in the one-tile-per-group kernel, the unit alternates between waiting
// for the tile's loads, transforming it, and storing it.  Here each work-group loops over
// tiles and keeps the next tile in flight in registers while the current one is
// transformed in LDS:
//
//   regs <- tile t0
//   loop: LDS <- pre-weighted regs; regs <- tile t+1 (no wait); FFT + post in LDS;
//         store tile t from LDS
//
// The transform itself (two real pencils packed in one complex FFT, symmetric
// pre-weighting, split + prefix sum) is the one of the single-tile kernels.  The tile
// shape is a compile-time constant, so the load/store index arithmetic folds to shifts,
// and the two pencils of a pair are adjacent columns, read and written as one 8-byte
// (FP32) or 16-byte (FP64) vector per position.  Requires an even column count per slab.
// Plain passes, the slowest-axis forward pass of the U-solve with eigen scaling and face
// sums, and (FP64) the whole slowest-axis Poisson pass (forward, scaling, inverse), whose
// prefetch is issued after the first transform.
#include "dst_device.h"

#include <algorithm>
#include <mutex>

namespace ahoc {

namespace fast {

namespace {

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

// Stage plan: 16 points per thread where a 16-point plan exists (N = 512, 1024), so that
// the prefetched tile fits in registers next to the transform's working set.
template <int N> using PipePlan = PlanOf<N, N == 512 || N == 1024>;

// Work-group size cap: 1024 (FP32) / 512 (FP64) threads for plans of at most 16 points per
// thread, 512 / 256 otherwise.
template <typename T, int N> constexpr int pipe_cap() {
  return PipePlan<N>::PPT <= 16 ? (sizeof(T) == 8 ? 512 : 1024) : (sizeof(T) == 8 ? 256 : 512);
}

// Pairs per work-group: 128-byte row segments (16 FP32 / 8 FP64 pairs), halved until the
// tile fits the size cap and 150 KB of LDS.
template <typename T, int N> constexpr int pipe_nseq() {
  constexpr int TPS = N / PipePlan<N>::PPT;
  constexpr int CAP = pipe_cap<T, N>();
  int nseq = sizeof(T) == 8 ? 8 : 16;
  while (nseq * TPS < 64) nseq *= 2;
  while (nseq > 1 && (nseq * TPS > CAP || (long long)nseq * seq_stride<N>() * 2 * (long long)sizeof(T) > 150 * 1024))
    nseq /= 2;
  return nseq;
}

// LDS of a tile (sequences and segment totals) and, in MODE 3, the face row and (where it
// fits) the per-position table after it
template <typename T, int N, int NSEQ> constexpr size_t pipe_tile_bytes() {
  constexpr int TPS = N / PipePlan<N>::PPT;
  return (size_t)(NSEQ * seq_stride<N>() + NSEQ * 2 * (TPS / 64 > 0 ? TPS / 64 : 1)) * sizeof(cx<T>);
}
constexpr size_t align16(size_t b) { return (b + 15) / 16 * 16; }
// Twiddles a transform reads: stage 2 (radix R1 over blocks of R0) reads exp(-2 pi i k / N) at
// r k N / (R0 R1), stage 3 (radix R2 over blocks of R0 R1) at r k, r < R, k < the block length
template <int N> constexpr int pipe_ntw() {
  using P = PipePlan<N>;
  int m = (P::R1 - 1) * (P::R0 - 1) * (N / (P::R0 * P::R1));
  if (P::S == 3 && (P::R2 - 1) * (P::R0 * P::R1 - 1) > m) m = (P::R2 - 1) * (P::R0 * P::R1 - 1);
  return (m + 2) & ~1;  // (entries 0..m, rounded to an even count)
}
// The transform's tile-invariant tables (those twiddles, and the pre-weighting sines
// sin(pi m / N), m <= N/2) in LDS after everything else, where it has room.  Read from global
// memory, they would be loads issued after the next tile's prefetch (and after the previous
// tile's stores), and a wavefront's memory operations complete in issue order: the first wait
// for a table value would also wait for the whole prefetch.
template <typename T, int N> constexpr size_t pipe_tab_bytes() {
  return align16((size_t)pipe_ntw<N>() * sizeof(cx<T>)) + align16((size_t)(N / 2 + 1) * sizeof(T));
}
// A load through a pointer chosen between two kernel arguments, kept in the global address
// space (a generic pointer would be a flat load, which the compiler waits for with every
// memory operation in flight)
template <typename T> __device__ __forceinline__ T gload(const T* p) {
  return *reinterpret_cast<const __attribute__((address_space(1))) T*>(reinterpret_cast<unsigned long long>(p));
}
// MODE 3 data after the tile: the face row (2 (N - 1) values) where it fits beside the
// transform tables (else it is read through the caches in the face loop: the tables take
// precedence), then the per-position table (4 (N - 1) values) where it fits
template <typename T, int N, int NSEQ> constexpr bool pipe_xrow_lds() {
  return align16(pipe_tile_bytes<T, N, NSEQ>() + 2 * (size_t)(N - 1) * sizeof(T)) + pipe_tab_bytes<T, N>() <=
             160 * 1024 ||
         align16(pipe_tile_bytes<T, N, NSEQ>()) + pipe_tab_bytes<T, N>() > 160 * 1024;
}
template <typename T, int N, int NSEQ, int MODE> constexpr size_t pipe_face_bytes() {
  return MODE == 3 && pipe_xrow_lds<T, N, NSEQ>() ? 2 * (size_t)(N - 1) * sizeof(T) : 0;
}
template <typename T, int N, int NSEQ, int MODE> constexpr bool pipe_tab_lds() {
  return align16(pipe_tile_bytes<T, N, NSEQ>() + pipe_face_bytes<T, N, NSEQ, MODE>()) + pipe_tab_bytes<T, N>() <=
         160 * 1024;
}
template <typename T, int N, int NSEQ> constexpr bool pipe_ptab_lds() {
  return align16(pipe_tile_bytes<T, N, NSEQ>() + 6 * (size_t)(N - 1) * sizeof(T)) +
             (pipe_tab_lds<T, N, NSEQ, 3>() ? pipe_tab_bytes<T, N>() : 0) <=
         160 * 1024;
}
// offset of the transform tables
template <typename T, int N, int NSEQ, int MODE> constexpr size_t pipe_tab_off() {
  return align16(pipe_tile_bytes<T, N, NSEQ>() + pipe_face_bytes<T, N, NSEQ, MODE>() +
                 (MODE == 3 && pipe_ptab_lds<T, N, NSEQ>() ? 4 * (size_t)(N - 1) * sizeof(T) : 0));
}
// MODES 1 and 2, after the transform tables where they fit: the eigenvalue sines of the pass
// axis (N - 1 values), then (MODE 1) the face-sum weights (2 (N - 1) values)
template <typename T, int N, int NSEQ, int MODE> constexpr bool pipe_stab_lds() {
  return (MODE == 1 || MODE == 2) && pipe_tab_lds<T, N, NSEQ, MODE>() &&
         pipe_tab_off<T, N, NSEQ, MODE>() + pipe_tab_bytes<T, N>() + align16((size_t)(N - 1) * sizeof(T)) <=
             160 * 1024;
}
template <typename T, int N, int NSEQ, int MODE> constexpr bool pipe_wtab_lds() {
  return MODE == 1 && pipe_stab_lds<T, N, NSEQ, MODE>() &&
         pipe_tab_off<T, N, NSEQ, MODE>() + pipe_tab_bytes<T, N>() + align16((size_t)(N - 1) * sizeof(T)) +
                 align16(2 * (size_t)(N - 1) * sizeof(T)) <=
             160 * 1024;
}
template <typename T, int N, int NSEQ, int MODE> constexpr size_t pipe_lds_bytes() {
  return pipe_tab_lds<T, N, NSEQ, MODE>()
             ? pipe_tab_off<T, N, NSEQ, MODE>() + pipe_tab_bytes<T, N>() +
                   (pipe_stab_lds<T, N, NSEQ, MODE>() ? align16((size_t)(N - 1) * sizeof(T)) : 0) +
                   (pipe_wtab_lds<T, N, NSEQ, MODE>() ? align16(2 * (size_t)(N - 1) * sizeof(T)) : 0)
             : pipe_tile_bytes<T, N, NSEQ>() + pipe_face_bytes<T, N, NSEQ, MODE>() +
                   (MODE == 3 && pipe_ptab_lds<T, N, NSEQ>() ? 4 * (size_t)(N - 1) * sizeof(T) : 0);
}

// NT: the volume is loaded and stored with the non-temporal policy (arrays larger than the
// caches, see NT_STORE_MIN_BYTES); a compile-time choice, so that the prefetched registers
// do not meet at a branch join, which would wait for the loads in flight.  NT launches also
// have whole tiles only (columns a multiple of the tile width), so their loads and stores
// have no ragged-tile branches: the next tile's sequences are written to LDS right after the
// current tile's stores, and the wait for the prefetched registers there leaves the stores
// in flight (a wavefront's memory operations complete in issue order, and a branch around
// the stores would make the compiler wait for them too).
template <typename T, int N, int NSEQ, int MODE, bool NT>
__global__ void __launch_bounds__(NSEQ*(N / PipePlan<N>::PPT)) k_dst_pipe(Args<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  using PL = PipePlan<N>;
  constexpr int PPT = PL::PPT;
  constexpr int TPS = N / PPT;
  constexpr int L = N - 1;
  constexpr int HN = N / 2;
  constexpr int U = PPT / 2;  // mirrored position pairs per thread and tile
  constexpr int LDQ = seq_stride<N>();
  constexpr int LGQ = ilog2(NSEQ);
  constexpr int NTOT = 2 * (TPS / 64 > 0 ? TPS / 64 : 1);
  static_assert((1 << LGQ) == NSEQ, "NSEQ must be a power of two");
  constexpr bool FULL = NT;  // whole tiles only (checked at launch)
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem);
  // The thread index and the table pointers pass through an empty asm statement at the top
  // of every tile, so that the compiler recomputes the (tile-invariant) LDS addresses and
  // twiddle loads inside the loop instead of hoisting them and holding them in registers.
  int tid;
  int s, ts, q, mi;
  cx<T>* seq;
  cx<T>* tot;
  auto remap = [&]() {
    tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    // transform mapping: pair s, lane ts within the pair
    s = tid / TPS;
    ts = tid - s * TPS;
    seq = lds + s * LDQ;
    tot = lds + NSEQ * LDQ + s * NTOT;
    // load/store mapping: pair q (fastest across lanes: one row segment per NSEQ lanes),
    // position offset mi
    q = tid & (NSEQ - 1);
    mi = tid >> LGQ;
  };
  remap();
  const long long inner = a.inner;
  const long long ntiles = a.outer * a.ntile_inner;
  // tile -> (slab o, first column c0 in the slab, MODE 3: row ib of the column decode), in
  // 32-bit arithmetic (tile counts and columns below 2^30, checked at launch); one decode per
  // tile, carried from the prefetch to the transform and the store
  struct TileAt {
    long long o, c0;
    unsigned ib;
  };
  auto at = [&](long long tile) {
    TileAt d;
    const unsigned t = (unsigned)tile, nti = (unsigned)a.ntile_inner;
    const unsigned ou = t / nti;
    const unsigned c0 = (t - ou * nti) * (unsigned)(2 * NSEQ);
    d.o = ou;
    d.c0 = c0;
    d.ib = MODE == 3 ? c0 / (unsigned)a.fs.na : 0u;
    return d;
  };
  // MODE 3: the tile's row of the face spectra normal to the fastest axis as (sum,
  // difference) pairs per position, in LDS after the tile (prefetched one tile ahead in
  // registers); then, where LDS has room, the per-position table (s, layer sine, face
  // weights), loaded once
  cx<T>* xrow = reinterpret_cast<cx<T>*>(smem + (size_t)(NSEQ * LDQ + NSEQ * NTOT) * sizeof(cx<T>));
  constexpr bool PTL = MODE == 3 && pipe_ptab_lds<T, N, NSEQ>();
  constexpr bool XLDS = MODE == 3 && pipe_xrow_lds<T, N, NSEQ>();
  cx<T>* ptl = xrow + L;  // [m - 1][2]
  if constexpr (PTL) {
    const cx<T>* pg = reinterpret_cast<const cx<T>*>(a.gn.ptab);
    for (int j = threadIdx.x; j < 2 * L; j += NSEQ * TPS) ptl[j] = pg[j];
  }
  constexpr bool TWL = pipe_tab_lds<T, N, NSEQ, MODE>();
  constexpr bool STL = pipe_stab_lds<T, N, NSEQ, MODE>();
  constexpr bool WTL = pipe_wtab_lds<T, N, NSEQ, MODE>();
  constexpr int NTW = pipe_ntw<N>();
  cx<T>* twl = reinterpret_cast<cx<T>*>(smem + pipe_tab_off<T, N, NSEQ, MODE>());
  T* snl = reinterpret_cast<T*>(smem + pipe_tab_off<T, N, NSEQ, MODE>() + align16((size_t)NTW * sizeof(cx<T>)));
  T* stl = reinterpret_cast<T*>(smem + pipe_tab_off<T, N, NSEQ, MODE>() + pipe_tab_bytes<T, N>());
  T* wtl = stl + align16((size_t)L * sizeof(T)) / sizeof(T);
  if constexpr (TWL) {
    for (int j = threadIdx.x; j < NTW; j += NSEQ * TPS) twl[j] = a.tw[j];
    for (int j = threadIdx.x; j <= HN; j += NSEQ * TPS) snl[j] = a.sn[j];
    if constexpr (STL)
      for (int j = threadIdx.x; j < L; j += NSEQ * TPS) stl[j] = a.fs.s_this[j];
    if constexpr (WTL)
      for (int j = threadIdx.x; j < 2 * L; j += NSEQ * TPS) wtl[j] = a.fc.w[j];
    __syncthreads();
  }
  const T* s_tab = STL ? stl : a.fs.s_this;
  const T* w_tab = WTL ? wtl : a.fc.w;
  constexpr int XR = MODE == 3 ? (L + NSEQ * TPS - 1) / (NSEQ * TPS) : 1;
  T xf[2][XR];
  auto xload = [&](const TileAt& d) {
    if constexpr (XLDS) {
      const T* la = a.gn.la + d.o * a.gn.aslab + (long long)d.ib * a.gn.arow;
      // (without a branch: positions past the row read its last one, unused)
#pragma unroll
      for (int r = 0; r < XR; ++r) {
        const int j0 = (int)threadIdx.x + r * NSEQ * TPS;
        const int j = j0 < L ? j0 : L - 1;
        xf[0][r] = la[(long long)j * a.gn.apitch];
        xf[1][r] = la[a.gn.aplane + (long long)j * a.gn.apitch];
      }
    }
  };

  cx<T> xr[U], yr[U];  // prefetched tile: positions m and N - m of both pencils
  auto tile_base = [&](const TileAt& d) { return d.o * (long long)L * inner + d.c0; };
  // Global accesses: each row of positions is a uniform 64-bit base (scalar registers) plus
  // a fixed per-lane 32-bit byte offset; the lanes of one access span at most TPS rows.
  const long long rowb = inner * (long long)sizeof(T);  // bytes from one position to the next
  const unsigned vlo = (unsigned)((2 * q + (long long)mi * inner) * (long long)sizeof(T));
  const unsigned vhi = (unsigned)((2 * q + (long long)(TPS - 1 - mi) * inner) * (long long)sizeof(T));
  auto load = [&](const TileAt& d) {
    const long long c0 = d.c0;
    const SBase src(a.in + tile_base(d));
    // columns past the slab (ragged last tile) read column 0 of the tile and are zeroed below
    const bool ok = FULL || c0 + 2 * q < inner;
    const unsigned dq = ok ? 0u : (unsigned)(2 * q * (int)sizeof(T));
    unsigned vl = vlo - dq, vh = vhi - dq;
    // keep the 32-bit offsets local to this block, so that each access is selected in the
    // scalar-base + 32-bit-offset form
    asm volatile("" : "+v"(vl), "+v"(vh));
    // position m - 1 = u TPS + mi; position N - m - 1 = (N - 1 - (u + 1) TPS) + (TPS - 1 - mi)
    // (for m = N/2 the latter is read but unused).  A volume larger than the caches streams
    // through once: non-temporal, so that it does not displace the tables and (MODE 3) the
    // re-read face spectra in L2
    if constexpr (NT) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        xr[u] = src.plus((long long)(u * TPS) * rowb).ld_nt<cx<T>>(vl);
        yr[u] = src.plus((long long)(N - 1 - (u + 1) * TPS) * rowb).ld_nt<cx<T>>(vh);
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        xr[u] = src.plus((long long)(u * TPS) * rowb).ld<cx<T>>(vl);
        yr[u] = src.plus((long long)(N - 1 - (u + 1) * TPS) * rowb).ld<cx<T>>(vh);
      }
    }
    if constexpr (!FULL) {
      if (c0 + 2 * NSEQ > inner && !ok) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          xr[u].x = xr[u].y = T(0);
          yr[u].x = yr[u].y = T(0);
        }
      }
    }
  };
  // positions m = 1 + mi + u TPS: with TPS a multiple of 32, one padded base per direction
  // plus immediate offsets (see poff)
  constexpr bool LIN = TPS % 32 == 0;
  auto to_lds = [&]() {
    cx<T>* sq = lds + q * LDQ;
    cx<T>* lo = sq + pad(1 + mi);
    cx<T>* hi = sq + pad(N - 1 - mi);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int m = 1 + mi + u * TPS;
      cx<T>* plo = LIN ? lo + poff(u * TPS) : sq + pad(m);
      cx<T>* phi = LIN ? hi - poff(u * TPS) : sq + pad(N - m);
      if (u == U - 1 && m == HN) {  // the middle position pairs with itself: 2 z
        cx<T> o;
        o.x = T(2) * xr[u].x;
        o.y = T(2) * xr[u].y;
        *plo = o;
      } else {
        const T w = TWL ? snl[m] : a.sn[m];
        const T sx = w * (xr[u].x + yr[u].x), sy = w * (xr[u].y + yr[u].y);
        const T dx = T(0.5) * (xr[u].x - yr[u].x), dy = T(0.5) * (xr[u].y - yr[u].y);
        cx<T> o1, o2;
        o1.x = sx + dx;
        o1.y = sy + dy;
        o2.x = sx - dx;
        o2.y = sy - dy;
        *plo = o1;
        *phi = o2;
      }
    }
    if (tid < NSEQ) {
      cx<T> z;
      z.x = T(0);
      z.y = T(0);
      lds[tid * LDQ] = z;
    }
  };
  auto store = [&](const TileAt& d) {
    const SBase dst(a.out + tile_base(d));
    if constexpr (!FULL) {
      if (d.c0 + 2 * q >= inner) return;
    }
    unsigned vs = vlo;
    asm volatile("" : "+v"(vs));
    const cx<T>* sq = lds + q * LDQ;
    const cx<T>* lo = sq + pad(1 + mi);
    if constexpr (NT) {
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const int m = 1 + mi + k * TPS;
        if (k < PPT - 1 || m < N)
          dst.plus((long long)(k * TPS) * rowb).st_nt<cx<T>>(vs, LIN ? lo[poff(k * TPS)] : sq[pad(m)]);
      }
    } else {
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const int m = 1 + mi + k * TPS;
        if (k < PPT - 1 || m < N)
          dst.plus((long long)(k * TPS) * rowb).st<cx<T>>(vs, LIN ? lo[poff(k * TPS)] : sq[pad(m)]);
      }
    }
  };

  // MODE 3: the face row of the tile from the prefetched registers, as (sum, difference)
  auto stage_x = [&]() {
    if constexpr (XLDS) {
#pragma unroll
      for (int r = 0; r < XR; ++r) {
        const int j = tid + r * NSEQ * TPS;
        if (j < L) {
          cx<T> xv;
          xv.x = xf[0][r] + xf[1][r];
          xv.y = xf[0][r] - xf[1][r];
          xrow[j] = xv;
        }
      }
    }
  };

  // MODE 3: the pair's per-tile coefficients (column sines, row sine, z-face pair at both
  // columns, face-layer weights), loaded without branches (indices clamped into the tables,
  // a missing table read at another's entry 0; the validity flags select where they are
  // used) at the top of the tile, before the next tile's prefetch: a wait for them does not
  // wait for the prefetch
  struct Coef3 {
    T saa, sab, sb, pa0, pa1, pb0, pb1, wla, wlb, wbl;
  };
  [[maybe_unused]] Coef3 c3;
  auto cload3 = [&](const TileAt& d) {
    if constexpr (MODE == 3) {
      const long long ca = d.c0 + 2 * s;
      const long long iaa = ca - (long long)d.ib * a.fs.na;
      const int ia = (int)(iaa < a.fs.nva ? iaa : a.fs.nva - 1);
      const int ia1 = (int)(iaa + 1 < a.fs.nva ? iaa + 1 : a.fs.nva - 1);
      const long long cc = ca < inner - 2 ? ca : inner - 2;
      const T* lp = a.gn.lp + d.o * a.gn.pslab;
      const T* sbp = a.fs.s_b ? a.fs.s_b + d.ib : a.fs.s_a;
      const T* wbp = a.gn.lb ? a.gn.wb + d.ib : a.gn.wa;
      c3.saa = a.fs.s_a[ia];
      c3.sab = a.fs.s_a[ia1];
      c3.sb = gload(sbp);
      c3.pa0 = lp[cc];
      c3.pa1 = lp[a.gn.pplane + cc];
      c3.pb0 = lp[cc + 1];
      c3.pb1 = lp[a.gn.pplane + cc + 1];
      c3.wla = a.gn.wa[ia];
      c3.wlb = a.gn.wa[ia1];
      c3.wbl = gload(wbp);
    }
  };

  // MODES 1 and 2: the pair's column and row sines, loaded the same way (a tile may span two
  // rows of the column decode here)
  struct Coef12 {
    T saa, sab, sba, sbb;
  };
  [[maybe_unused]] Coef12 c12;
  auto cload12 = [&](const TileAt& d) {
    if constexpr (MODE == 1 || MODE == 2) {
      const long long ca = d.c0 + 2 * s;
      auto one = [&](long long col, T& sa, T& sb) {
        const unsigned cc = (unsigned)(col < inner ? col : inner - 1);
        const unsigned ib = cc / (unsigned)a.fs.na;
        const unsigned ia = cc - ib * (unsigned)a.fs.na;
        sa = a.fs.s_a[ia < (unsigned)a.fs.nva ? ia : (unsigned)a.fs.nva - 1];
        sb = gload(a.fs.s_b ? a.fs.s_b + ib : a.fs.s_a);
      };
      one(ca, c12.saa, c12.sba);
      one(ca + 1, c12.sab, c12.sbb);
    }
  };

  long long tile = blockIdx.x;
  TileAt cur = at(tile);
  if (tile < ntiles) {
    load(cur);
    xload(cur);
    to_lds();
    stage_x();
  }
  for (; tile < ntiles; tile += gridDim.x) {
    remap();
    const cx<T>* tw = TWL ? twl : a.tw;
    __syncthreads();  // the tile's sequences (and face row) in LDS
    cload3(cur);
    cload12(cur);
    const long long nxt = tile + gridDim.x;
    // the next tile is in flight during the transform below (with two transforms, during
    // the second one only: the prefetched registers are not live across both).  The last
    // tile of a work-group prefetches itself (unused): a prefetch without a branch, so that
    // waits for loads issued before it are not taken as waits for it
    const TileAt nd = at(nxt < ntiles ? nxt : tile);
    if constexpr (MODE != 2) {
      load(nd);
      xload(nd);
    }

    cx<T> A, B;
    A.x = A.y = T(1);
    B.x = B.y = T(0);
    fft<T, N, PL>(seq, ts, tw);
    if constexpr (MODE != 0) {
      // forward transform of the slowest axis and eigen scaling; then either the face sums
      // of the scaled spectrum along the pass axis per column (MODE 1: the scaled spectrum
      // itself is the output) or the inverse transform (MODE 2: a whole Poisson pass)
      const long long o = cur.o;
      const long long c0 = cur.c0;
      const long long ca = c0 + 2 * s, cb = ca + 1;
      if constexpr (MODE == 3) {
        const long long iaa = ca - (long long)cur.ib * a.fs.na;
        const T sb = a.fs.s_b ? c3.sb : T(0);
        auto coef3 = [&](bool v, T sa, T& Ao, T& Bo) {
          Ao = v ? sa + sb + a.fs.c_ab * sa * sb + (a.fs.a0 + a.fs.ka * sa + a.fs.kb * sb) : T(1);
          Bo = v ? T(1) + a.fs.c_ta * sa + a.fs.c_tb * sb + a.fs.kt : T(0);
        };
        coef3(ca < inner && iaa < a.fs.nva, c3.saa, A.x, B.x);
        coef3(cb < inner && iaa + 1 < a.fs.nva, c3.sab, A.y, B.y);
      } else {
        // the prefetched sines, selected by the column's validity
        auto coef12 = [&](long long col, T sa, T sbv, T& Ao, T& Bo) {
          const unsigned ib = (unsigned)col / (unsigned)a.fs.na;  // col < inner < 2^31
          const long long ia = col - (long long)ib * a.fs.na;
          const bool v = col < inner && ia < a.fs.nva;
          const T sb = a.fs.s_b ? sbv : T(0);
          Ao = v ? sa + sb + a.fs.c_ab * sa * sb + (a.fs.a0 + a.fs.ka * sa + a.fs.kb * sb) : T(1);
          Bo = v ? T(1) + a.fs.c_ta * sa + a.fs.c_tb * sb + a.fs.kt : T(0);
        };
        coef12(ca, c12.saa, c12.sba, A.x, B.x);
        coef12(cb, c12.sab, c12.sbb, A.y, B.y);
      }
      // MODE 3 scales in the face loop below, after adding the face-layer term
      if constexpr (MODE == 3) post<T, N, PL, false>(seq, tot, ts, A, B, nullptr, T(0));
      else post<T, N, PL, true>(seq, tot, ts, A, B, s_tab, a.fs.scale);
      if constexpr (MODE == 2) {
        load(nd);
        pre_lds<T, N, PL>(seq, ts, TWL ? snl : a.sn);
        fft<T, N, PL>(seq, ts, tw);
        A.x = A.y = T(1);
        B.x = B.y = T(0);
        post<T, N, PL, false>(seq, tot, ts, A, B, nullptr, T(0));
      } else {
      T la = 0, ha = 0, lb = 0, hb = 0;
      // MODE 3: U = scale (mu_M W + G) / lambda_L at (column, position m), with the
      // symbol of the weighting operator mu_M = Ca + D s (pencil a), Cb + D s (pencil b) and
      // G the face-layer source's spectrum: one face value times one layer sine per face
      // pair (faces as sums/differences, selected by the parity of the mode across the
      // face; see k_gen_pipe)
      [[maybe_unused]] T ga0 = 0, gb0 = 0, wla = 0, wlb = 0, wbl = 0, Ca = 1, Cb = 1, D = 0;
      // y-face values of the pair at position m (face spectra stored [side][column][position],
      // so the lanes of a pair read consecutive positions): the face plane of the mode's
      // parity as a uniform base, the pair's two rows as 32-bit offsets
      [[maybe_unused]] const T* ybase = nullptr;
      [[maybe_unused]] unsigned yoff = 0, ystep = 0;
      // MODE 3: the tile lies in row ib of the column decode (na a multiple of the tile
      // width, checked at launch), so the pair's columns are iaa and iaa + 1 of that row
      [[maybe_unused]] const long long ib = cur.ib;
      [[maybe_unused]] const long long iaa = ca - ib * a.fs.na;
      [[maybe_unused]] const bool va = MODE == 3 && ca < inner && iaa < a.fs.nva;
      [[maybe_unused]] const bool vb = MODE == 3 && cb < inner && iaa + 1 < a.fs.nva;
      if constexpr (MODE == 3) {
        // every position of this thread has the parity of 1 + ts (TPS is even)
        const bool modd = ((1 + ts) & 1) != 0;
        // z-face pair as its sum (odd mode) or difference (even mode)
        const T sg = modd ? T(1) : T(-1);
        ga0 = va ? c3.pa0 + sg * c3.pa1 : T(0);
        gb0 = vb ? c3.pb0 + sg * c3.pb1 : T(0);
        wla = va ? c3.wla : T(0);
        wlb = vb ? c3.wlb : T(0);
        // y faces: without them the loads below read the per-position table (any array of at
        // least N values) with weight zero, so that the face loop has no branch
        if (a.gn.lb) {
          wbl = c3.wbl;
          ybase = a.gn.lb + o * a.gn.bslab + ((ib & 1) ? a.gn.bplane : 0);
          yoff = (unsigned)((iaa * a.gn.bpitch + ts) * (long long)sizeof(T));
          ystep = (unsigned)(a.gn.bpitch * (long long)sizeof(T));
        } else {
          wbl = T(0);
          ybase = a.gn.ptab;
          yoff = (unsigned)(ts * (int)sizeof(T));
          ystep = 0;
        }
        const T sb = a.fs.s_b ? c3.sb : T(0);
        Ca = va ? a.fs.mc0 + a.fs.mca * c3.saa + a.fs.mcb * sb : T(1);
        Cb = vb ? a.fs.mc0 + a.fs.mca * c3.sab + a.fs.mcb * sb : T(1);
        D = a.fs.mct;
      }
      if constexpr (MODE == 3) {
        // groups of G positions: the group's table and y-face loads are all issued before
        // its arithmetic (a scheduling barrier keeps the compiler from interleaving them,
        // which it otherwise does to save registers, one load round trip per position).
        // Positions past the transform (the last thread's last one) read position N - 1.
        constexpr int G = N >= 2048 ? 2 : 4;  // (longer transforms hold more registers)
        static_assert(PPT % G == 0, "whole groups of positions");
        const cx<T>* ptb = PTL ? ptl : reinterpret_cast<const cx<T>*>(a.gn.ptab);
        const SBase ys(ybase);  // byte offsets below 2^32 (checked at launch)
        // the tile's x-face row, where it is not in LDS
        [[maybe_unused]] const T* xla = a.gn.la + o * a.gn.aslab + ib * a.gn.arow;
#pragma unroll 1
        for (int i0 = 0; i0 < PPT; i0 += G) {
          cx<T> t0[G], t1[G];
          T y0[G], y1[G];
          [[maybe_unused]] T x0[G], x1[G];
#pragma unroll
          for (int g = 0; g < G; ++g) {
            const int m = 1 + ts + (i0 + g) * TPS;
            const int mc = m < N ? m : N - 1;
            t0[g] = ptb[2 * (mc - 1)];
            t1[g] = ptb[2 * (mc - 1) + 1];
            if constexpr (!XLDS) {
              x0[g] = xla[(long long)(mc - 1) * a.gn.apitch];
              x1[g] = xla[a.gn.aplane + (long long)(mc - 1) * a.gn.apitch];
            }
            const unsigned off = yoff + (unsigned)((mc - 1 - ts) * (int)sizeof(T));
            y0[g] = ys.template ld<T>(off);
            y1[g] = ys.template ld<T>(off + ystep);
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int g = 0; g < G; ++g) {
            const int i = i0 + g;
            const int m = 1 + ts + i * TPS;
            if (i < PPT - 1 || m < N) {
              cx<T>* pv = LIN ? seq + pad(1 + ts) + poff(i * TPS) : seq + pad(m);
              cx<T> v = *pv;
              const T st = t0[g].x, wpl = t0[g].y;
              cx<T> xv;  // the x-face pair as (sum, difference)
              if constexpr (XLDS) {
                xv = xrow[m - 1];
              } else {
                xv.x = x0[g] + x1[g];
                xv.y = x0[g] - x1[g];
              }
              const T ga = ga0 * wpl + xv.x * wla + y0[g] * wbl;
              const T gb = gb0 * wpl + xv.y * wlb + y1[g] * wbl;
              v.x = (v.x * (Ca + D * st) + (va ? ga : T(0))) * (a.fs.scale * recip(A.x + B.x * st));
              v.y = (v.y * (Cb + D * st) + (vb ? gb : T(0))) * (a.fs.scale * recip(A.y + B.y * st));
              *pv = v;
              const T wl = t1[g].x, wh = t1[g].y;
              la += v.x * wl;
              ha += v.x * wh;
              lb += v.y * wl;
              hb += v.y * wh;
            }
          }
          __builtin_amdgcn_sched_barrier(0);  // (the next group's loads after this one)
        }
      } else {
#pragma unroll
      for (int i = 0; i < PPT; ++i) {
        const int m = 1 + ts + i * TPS;
        if (i < PPT - 1 || m < N) {
          cx<T>* pv = LIN ? seq + pad(1 + ts) + poff(i * TPS) : seq + pad(m);
          const cx<T> v = *pv;
          const T wl = w_tab[m - 1], wh = w_tab[L + m - 1];
          la += v.x * wl;
          ha += v.x * wh;
          lb += v.y * wl;
          hb += v.y * wh;
        }
      }
      }
      seg_sum4<T, TPS>(la, ha, lb, hb, tot, ts);
      if (ts == 0) {
        T* fo = a.fc.out + o * a.fc.slab;
        if (ca < inner) {
          fo[ca] = la;
          fo[a.fc.plane + ca] = ha;
        }
        if (cb < inner) {
          fo[cb] = lb;
          fo[a.fc.plane + cb] = hb;
        }
      }
      }
    } else {
      post<T, N, PL, false>(seq, tot, ts, A, B, nullptr, T(0));
    }
    __syncthreads();  // the store reads other pairs' sequences
    store(cur);
    __syncthreads();  // the next tile overwrites LDS
    if (nxt < ntiles) {
      to_lds();
      stage_x();
    }
    cur = nd;
  }
}

template <typename T, int N, int MODE> struct PipeLaunch {
  static constexpr int NSEQ = pipe_nseq<T, N>();
  static constexpr int TPS = N / PipePlan<N>::PPT;
  static constexpr int THREADS = NSEQ * TPS;
  static constexpr size_t LDS = pipe_lds_bytes<T, N, NSEQ, MODE>();

  // the non-temporal form exists where a volume can exceed the caches (N >= 384)
  static constexpr bool HAS_NT = N >= 384;

  // resident work-groups on the device (persistent grid)
  template <bool NT> static int resident() {
    static std::once_flag once;
    static int r = 0;
    std::call_once(once, [] {
      const void* fn = reinterpret_cast<const void*>(&k_dst_pipe<T, N, NSEQ, MODE, NT && HAS_NT>);
      (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      int dev = 0, cus = 0, per = 0;
      if (hipGetDevice(&dev) == hipSuccess &&
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
          hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, THREADS, LDS) == hipSuccess && per > 0)
        r = cus * per;
      (void)hipGetLastError();
    });
    return r;
  }

  static int run(Args<T>& a, int nseq, hipStream_t st) {
    if (nseq > 0 && nseq != NSEQ) return ST_UNSUPPORTED;
    if (THREADS % 64 != 0 || THREADS > pipe_cap<T, N>() || LDS > 160 * 1024) return ST_UNSUPPORTED;
    // per-lane byte offsets span TPS rows and must fit in 32 bits
    if ((double)(TPS + 1) * (double)a.inner * (double)sizeof(T) >= 4294967295.0) return ST_UNSUPPORTED;
    // (the non-temporal form takes whole tiles only)
    const bool nt = HAS_NT && a.inner % (2 * NSEQ) == 0 &&
                    (double)a.outer * (double)a.inner * (double)(N - 1) * sizeof(T) >= NT_STORE_MIN_BYTES;
    const int res = nt ? resident<true>() : resident<false>();
    if (res <= 0) return ST_UNSUPPORTED;
    a.lg_nseq = ilog2(NSEQ);
    a.ntile_inner = (a.inner + 2LL * NSEQ - 1) / (2LL * NSEQ);
    a.ntst = nt;
    const long long ntiles = a.outer * a.ntile_inner;
    if (ntiles <= 0) return ST_OK;
    // the kernel decodes tiles and columns in 32-bit arithmetic
    if (a.inner >= (1LL << 30) || ntiles >= (1LL << 30)) return ST_UNSUPPORTED;
    if (MODE == 3 && (a.fs.na <= 0 || a.fs.na % (2 * NSEQ) != 0)) return ST_UNSUPPORTED;
    const long long grid = ntiles < res ? ntiles : res;
    if (nt)
      hipLaunchKernelGGL((k_dst_pipe<T, N, NSEQ, MODE, HAS_NT>), dim3((unsigned)grid), dim3(THREADS), LDS, st, a);
    else
      hipLaunchKernelGGL((k_dst_pipe<T, N, NSEQ, MODE, false>), dim3((unsigned)grid), dim3(THREADS), LDS, st, a);
    AHOC_HIP_TRY(hipGetLastError());
    return ST_OK;
  }
};

// ------------------------------------------------------------------------------------
// Persistent V-solve pass along the slowest axis: generate the scaled spectrum of the
// face-layer right-hand side from the 2-D face spectra (see dst_spectral.hip for the
// separable form), invert along the pass axis, store.  Same tile mapping as k_dst_pipe.
// Face-array layouts as DstGen (common.h); a tile must lie in one row of the column decode
// (na a multiple of the tile width), so that the x-face row is shared by all its columns.
//
// Mode k of the layer next to the high face carries the layer sine of the low face times
// (-1)^(k+1) (sin(pi k (N-1)/N)), so a face pair enters mode k only through lo + hi (k odd)
// or lo - hi (k even).  The x- and z-face pairs are combined where they are read (two
// loads per tile and column); the y-face pairs, read at every position, are turned into
// their sum and difference in place by k_face_pm first.  Then a term is one face value
// times one layer sine:
//   z faces  P(kx, ky) at the position parity of the pass axis (fixed per thread, since a
//            thread's positions are TPS apart and TPS is even)
//   x faces  X(ky, kz): the pair's even column (odd mode) the sum, its odd column the
//            difference; one row per tile, staged in LDS
//   y faces  Y(kx, kz) at the parity of ky (fixed per tile); prefetched into registers
//            for the next tile while the current one is transformed
// The layer sines and eigenvalue tables of the pass axis are tile-invariant: LDS where
// it has room, else registers (512-thread groups) or the caches.
// ------------------------------------------------------------------------------------
template <typename T> struct GenPipeArgs {
  T* out;
  const cx<T>* tw;
  const T* sn;
  long long outer, inner, ntile_inner;
  DstScale<T> fs;
  DstGen<T> g;
};

// (lo, hi) -> (lo + hi, lo - hi) for `count` entries of each of `nslab` slabs:
// lo = f[o slab + j], hi = f[o slab + plane + j]
template <typename T>
__global__ void k_face_pm(T* f, long long plane, long long slab, long long count, long long nslab) {
  const long long n = count * nslab;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const long long o = e / count;
    const long long j = e - o * count;
    T* lo = f + o * slab + j;
    const T a = lo[0], b = lo[plane];
    lo[0] = a + b;
    lo[plane] = a - b;
  }
}

template <typename T> int face_pm(T* f, long long plane, long long slab, long long count, long long nslab, hipStream_t st) {
  if (!f || count <= 0 || nslab <= 0) return ST_OK;
  const long long n = count * nslab;
  const unsigned blocks = (unsigned)std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL((k_face_pm<T>), dim3(blocks), dim3(256), 0, st, f, plane, slab, count, nslab);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

template <typename T, int N, int NSEQ> struct GenShape {
  using PL = PipePlan<N>;
  static constexpr int PPT = PL::PPT;
  static constexpr int TPS = N / PPT;
  static constexpr int L = N - 1;
  static constexpr int THREADS = NSEQ * TPS;
  static constexpr int NTOT = 2 * (TPS / 64 > 0 ? TPS / 64 : 1);
  static constexpr size_t TILE_B = (size_t)(NSEQ * seq_stride<N>() + NSEQ * NTOT) * sizeof(cx<T>);
  static constexpr size_t LDS_MAX = 160 * 1024;
  // x-face row as (sum, difference) per position in LDS; then the tables as (layer sine,
  // eigenvalue) per position
  static constexpr bool XLDS = TILE_B + 2 * (size_t)L * sizeof(T) <= LDS_MAX;
  static constexpr bool TLDS = XLDS && TILE_B + 4 * (size_t)L * sizeof(T) <= LDS_MAX;
  static constexpr int XR = (L + THREADS - 1) / THREADS;  // x-face entries per thread and side
  static constexpr size_t BASE = TILE_B + (XLDS ? 2 * (size_t)L * sizeof(T) : 0) + (TLDS ? 2 * (size_t)L * sizeof(T) : 0);
  // then the transform's twiddles and pre-weighting sines (as in k_dst_pipe), where they fit
  static constexpr size_t TAB_OFF = align16(BASE);
  static constexpr bool TWL = TAB_OFF + pipe_tab_bytes<T, N>() <= LDS_MAX;
  static constexpr size_t LDS = TWL ? TAB_OFF + pipe_tab_bytes<T, N>() : BASE;
};

// NT: non-temporal stores and whole tiles only (as in k_dst_pipe)
template <typename T, int N, int NSEQ, bool NT>
__global__ void __launch_bounds__(NSEQ*(N / PipePlan<N>::PPT)) k_gen_pipe(GenPipeArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  using SH = GenShape<T, N, NSEQ>;
  using PL = typename SH::PL;
  constexpr int PPT = SH::PPT;
  constexpr int TPS = SH::TPS;
  constexpr int L = SH::L;
  constexpr int HN = N / 2;
  constexpr int U = PPT / 2;
  constexpr int THREADS = SH::THREADS;
  constexpr int LDQ = seq_stride<N>();
  constexpr int LGQ = ilog2(NSEQ);
  constexpr int NTOT = SH::NTOT;
  constexpr bool LIN = TPS % 32 == 0;
  constexpr bool XLDS = SH::XLDS, TLDS = SH::TLDS;
  constexpr int XR = SH::XR;
  constexpr bool FULL = NT;  // whole tiles only (checked at launch)
  static_assert(TPS % 2 == 0, "positions of a thread must share their parity");
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem);
  cx<T>* xrow = reinterpret_cast<cx<T>*>(smem + SH::TILE_B);  // (sum, difference) per position
  cx<T>* tab = xrow + L;                                       // (layer sine, eigenvalue) per position
  constexpr bool TWL = SH::TWL;
  constexpr int NTW = pipe_ntw<N>();
  cx<T>* twl = reinterpret_cast<cx<T>*>(smem + SH::TAB_OFF);
  T* snl = reinterpret_cast<T*>(smem + SH::TAB_OFF + align16((size_t)NTW * sizeof(cx<T>)));
  const long long inner = a.inner;
  const long long ntiles = a.outer * a.ntile_inner;
  const DstGen<T>& g = a.g;
  const bool has_b = g.lb != nullptr;

  const int tid0 = threadIdx.x;
  const int q0 = tid0 & (NSEQ - 1);
  const int mi0 = tid0 >> LGQ;
  // the thread's positions m = 1 + mi + u TPS and N - m all have the parity of 1 + mi
  const bool modd = ((1 + mi0) & 1) != 0;

  // tile-invariant tables of the pass axis
  if constexpr (TLDS) {
    for (int j = tid0; j < L; j += THREADS) {
      cx<T> t;
      t.x = g.wp[j];
      t.y = a.fs.s_this[j];
      tab[j] = t;
    }
  }
  if constexpr (TWL) {
    for (int j = tid0; j < NTW; j += THREADS) twl[j] = a.tw[j];
    for (int j = tid0; j <= HN; j += THREADS) snl[j] = a.sn[j];
  }

  // tile -> (slab o, first column c0 in the slab, row ib of the column decode), in 32-bit
  // arithmetic (tile counts and columns below 2^30, checked at launch); one decode per tile,
  // carried from the prefetch to the generation and the store
  struct TileAt {
    long long o, c0, ib;
  };
  auto at = [&](long long tile) {
    TileAt d;
    const unsigned t = (unsigned)tile, nti = (unsigned)a.ntile_inner;
    const unsigned ou = t / nti;
    const unsigned c0 = (t - ou * nti) * (unsigned)(2 * NSEQ);
    d.o = ou;
    d.c0 = c0;
    d.ib = c0 / (unsigned)a.fs.na;
    return d;
  };
  // prefetched face data of a tile: the y-face values at the thread's mirrored positions
  // (both pencils of its pair) and the tile's x-face row
  cx<T> ylo[U], yhi[U];
  T xr[2][XR];
  const long long rowb = (long long)g.bpitch * (long long)sizeof(T);
  auto prefetch = [&](const TileAt& d) {
    const long long o = d.o, c0 = d.c0, ib = d.ib;
    if (has_b) {
      const long long ia0 = c0 - ib * a.fs.na;  // first column of the tile in its row
      // ky even (odd mode) -> sums, ky odd -> differences
      const T* yrow = g.lb + o * g.bslab + ((ib & 1) ? g.bplane : 0) + ia0;
      const SBase src(yrow);
      unsigned vlo = (unsigned)((2 * q0 + (long long)mi0 * g.bpitch) * (long long)sizeof(T));
      unsigned vhi = (unsigned)((2 * q0 + (long long)(TPS - 1 - mi0) * g.bpitch) * (long long)sizeof(T));
      asm volatile("" : "+v"(vlo), "+v"(vhi));
#pragma unroll
      for (int u = 0; u < U; ++u) {
        // position m - 1 = u TPS + mi; position N - m - 1 = (N - 1 - (u + 1) TPS) + (TPS - 1 - mi)
        ylo[u] = src.plus((long long)(u * TPS) * rowb).ld<cx<T>>(vlo);
        yhi[u] = src.plus((long long)(N - 1 - (u + 1) * TPS) * rowb).ld<cx<T>>(vhi);
      }
    }
    if constexpr (XLDS) {
      const T* la = g.la + o * g.aslab + ib * g.arow;
#pragma unroll
      for (int r = 0; r < XR; ++r) {
        const int j = tid0 + r * THREADS;
        if (j < L) {
          xr[0][r] = la[(long long)j * g.apitch];
          xr[1][r] = la[g.aplane + (long long)j * g.apitch];
        }
      }
    }
  };

  // per-tile coefficients, prefetched with the face data (loads issued before the stores
  // of the tile in flight): the pair's column sines, the row sine, the z-face pair at both
  // columns, the layer weights of the x and y faces.  Indices clamped into the tables; the
  // validity flags select the values where they are used.
  struct Coef {
    T saa, sab, sb, pa0, pa1, pb0, pb1, wla, wlb, wbl;
  };
  Coef cf;
  auto cload = [&](const TileAt& d) {
    const long long ca = d.c0 + 2 * q0;
    const int iaa = (int)(ca - d.ib * a.fs.na);
    const int ia = iaa < a.fs.nva ? iaa : a.fs.nva - 1;
    const int ib_ = iaa + 1 < a.fs.nva ? iaa + 1 : a.fs.nva - 1;
    const long long cc = ca < inner - 2 ? ca : inner - 2;
    const T* lp = g.lp + d.o * g.pslab;
    cf.saa = a.fs.s_a[ia];
    cf.sab = a.fs.s_a[ib_];
    // (loads without a branch: a missing table reads entry 0 of another and is zeroed where used)
    cf.sb = gload(a.fs.s_b ? a.fs.s_b + d.ib : a.fs.s_a);
    cf.pa0 = lp[cc];
    cf.pa1 = lp[g.pplane + cc];
    cf.pb0 = lp[cc + 1];
    cf.pb1 = lp[g.pplane + cc + 1];
    cf.wla = g.wa[ia];
    cf.wlb = g.wa[ib_];
    cf.wbl = gload(has_b ? g.wb + d.ib : g.wa);
  };

  // Generate the scaled spectrum of tile d into LDS and pre-weight it for the inverse
  // transform, from the prefetched registers
  auto generate = [&](const TileAt& d) {
    // thread index through an empty asm: tile-invariant addresses stay inside the loop
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int q = tid & (NSEQ - 1);
    const int mi = tid >> LGQ;
    const long long o = d.o;  // slab (instance of a batch)
    const long long c0 = d.c0;
    // ---- per pair: column decode, eigenvalue coefficients (divided by the scale), face values
    const long long ib = d.ib;  // one row per tile
    const long long ca = c0 + 2 * q;
    const int iaa = (int)(ca - ib * a.fs.na), iab = iaa + 1;
    const bool va = ca < inner && iaa < a.fs.nva, vb = ca + 1 < inner && iab < a.fs.nva;
    const T sb = a.fs.s_b ? cf.sb : T(0);
    const T isc = T(1) / a.fs.scale;
    T Aa = 1, Ba = 0, Ab = 1, Bb = 0;
    if (va) {
      const T sa = cf.saa;
      Aa = (sa + sb + a.fs.c_ab * sa * sb + (a.fs.a0 + a.fs.ka * sa + a.fs.kb * sb)) * isc;
      Ba = (T(1) + a.fs.c_ta * sa + a.fs.c_tb * sb + a.fs.kt) * isc;
    }
    if (vb) {
      const T sa = cf.sab;
      Ab = (sa + sb + a.fs.c_ab * sa * sb + (a.fs.a0 + a.fs.ka * sa + a.fs.kb * sb)) * isc;
      Bb = (T(1) + a.fs.c_ta * sa + a.fs.c_tb * sb + a.fs.kt) * isc;
    }
    // z-face pair as its sum (odd mode) or difference (even mode)
    const T sg = modd ? T(1) : T(-1);
    const T pa = va ? cf.pa0 + sg * cf.pa1 : T(0), pb = vb ? cf.pb0 + sg * cf.pb1 : T(0);
    const T wla = va ? cf.wla : T(0), wlb = vb ? cf.wlb : T(0);
    const T wbl = has_b ? cf.wbl : T(0);
    const T* la = g.la + o * g.aslab + ib * g.arow;
    if constexpr (XLDS) {
#pragma unroll
      for (int r = 0; r < XR; ++r) {
        const int j = tid + r * THREADS;
        if (j < L) {
          cx<T> xv;  // the face pair as (sum, difference)
          xv.x = xr[0][r] + xr[1][r];
          xv.y = xr[0][r] - xr[1][r];
          xrow[j] = xv;
        }
      }
    }
    __syncthreads();  // x-face row (and, first time round, the tables) visible
    // ---- generate the scaled spectrum at the mirrored positions m, N - m of pair q and
    // pre-weight them for the inverse transform: w_m = s_m (z_m + z_{N-m}) + (z_m - z_{N-m}) / 2
    auto gen_at = [&](int m, const cx<T>& y, T& ga, T& gb) {
      T wpl, st, xa, xb;
      if constexpr (TLDS) {
        const cx<T> t = tab[m - 1];
        wpl = t.x;
        st = t.y;
      } else {
        wpl = g.wp[m - 1];
        st = a.fs.s_this[m - 1];
      }
      if constexpr (XLDS) {
        const cx<T> xv = xrow[m - 1];
        xa = xv.x;
        xb = xv.y;
      } else {
        const T lo = la[(long long)(m - 1) * g.apitch], hi = la[g.aplane + (long long)(m - 1) * g.apitch];
        xa = lo + hi;
        xb = lo - hi;
      }
      ga = pa * wpl + xa * wla;
      gb = pb * wpl + xb * wlb;
      if (has_b) {
        ga += y.x * wbl;
        gb += y.y * wbl;
      }
      ga = va ? ga * recip(Aa + Ba * st) : T(0);
      gb = vb ? gb * recip(Ab + Bb * st) : T(0);
    };
    cx<T>* sq = lds + q * LDQ;
    cx<T>* lo = sq + pad(1 + mi);
    cx<T>* hi = sq + pad(N - 1 - mi);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int m = 1 + mi + u * TPS;
      cx<T>* plo = LIN ? lo + poff(u * TPS) : sq + pad(m);
      cx<T>* phi = LIN ? hi - poff(u * TPS) : sq + pad(N - m);
      T xa, xb;
      gen_at(m, ylo[u], xa, xb);
      if (u == U - 1 && m == HN) {  // the middle position pairs with itself: 2 z
        cx<T> v;
        v.x = T(2) * xa;
        v.y = T(2) * xb;
        *plo = v;
      } else {
        T ya, yb;
        gen_at(N - m, yhi[u], ya, yb);
        const T w = TWL ? snl[m] : a.sn[m];
        const T sx = w * (xa + ya), sy = w * (xb + yb);
        const T dx = T(0.5) * (xa - ya), dy = T(0.5) * (xb - yb);
        cx<T> o1, o2;
        o1.x = sx + dx;
        o1.y = sy + dy;
        o2.x = sx - dx;
        o2.y = sy - dy;
        *plo = o1;
        *phi = o2;
      }
    }
    if (tid < NSEQ) {
      cx<T> z;
      z.x = T(0);
      z.y = T(0);
      lds[tid * LDQ] = z;
    }
  };

  // Loop order: the tile's spectrum is generated at the end of the previous iteration,
  // after that tile's stores, from registers prefetched before its transform; with whole
  // tiles (FULL) the stores have no branch, so the wait for the prefetched registers there
  // leaves the stores in flight (memory operations complete in issue order).
  long long tile = blockIdx.x;
  TileAt cur = at(tile);
  if (tile < ntiles) {
    prefetch(cur);
    cload(cur);
    generate(cur);
  }
  for (; tile < ntiles; tile += gridDim.x) {
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int q = tid & (NSEQ - 1);
    const int mi = tid >> LGQ;
    __syncthreads();  // the tile's generated sequences in LDS
    // the next tile's face data is in flight during the transform below (the last tile of
    // a work-group prefetches itself, unused: no branch around the prefetch)
    const long long nxt = tile + gridDim.x;
    const TileAt nd = at(nxt < ntiles ? nxt : tile);
    prefetch(nd);
    cload(nd);
    // ---- inverse transform along the pass axis
    const int s = tid / TPS;
    const int ts = tid - s * TPS;
    cx<T>* seq = lds + s * LDQ;
    cx<T>* tot = lds + NSEQ * LDQ + s * NTOT;
    cx<T> A, B;
    A.x = A.y = T(1);
    B.x = B.y = T(0);
    fft<T, N, PL>(seq, ts, TWL ? twl : a.tw);
    post<T, N, PL, false>(seq, tot, ts, A, B, nullptr, T(0));
    __syncthreads();  // the store reads other pairs' sequences
    // ---- store (uniform row bases, fixed per-lane byte offsets)
    if (FULL || cur.c0 + 2 * q < inner) {
      const long long orowb = inner * (long long)sizeof(T);
      const SBase dst(a.out + cur.o * (long long)L * inner + cur.c0);
      unsigned vs = (unsigned)((2 * q + (long long)mi * inner) * (long long)sizeof(T));
      asm volatile("" : "+v"(vs));
      const cx<T>* sq = lds + q * LDQ;
      const cx<T>* lo = sq + pad(1 + mi);
      if constexpr (NT) {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          const int m = 1 + mi + k * TPS;
          if (k < PPT - 1 || m < N)
            dst.plus((long long)(k * TPS) * orowb).st_nt<cx<T>>(vs, LIN ? lo[poff(k * TPS)] : sq[pad(m)]);
        }
      } else {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          const int m = 1 + mi + k * TPS;
          if (k < PPT - 1 || m < N)
            dst.plus((long long)(k * TPS) * orowb).st<cx<T>>(vs, LIN ? lo[poff(k * TPS)] : sq[pad(m)]);
        }
      }
    }
    // the next tile's generation first stages its x-face row (a region the stores do not
    // read), then waits at its own barrier before it overwrites the sequences
    if (nxt < ntiles) generate(nd);
    cur = nd;
  }
}

template <typename T, int N> struct GenPipeLaunch {
  static constexpr int NSEQ = pipe_nseq<T, N>();
  static constexpr int TPS = N / PipePlan<N>::PPT;
  static constexpr int THREADS = NSEQ * TPS;
  static constexpr size_t LDS = GenShape<T, N, NSEQ>::LDS;
  // the non-temporal form exists where a volume can exceed the caches (N >= 384)
  static constexpr bool HAS_NT = N >= 384;

  template <bool NT> static int resident() {
    static std::once_flag once;
    static int r = 0;
    std::call_once(once, [] {
      const void* fn = reinterpret_cast<const void*>(&k_gen_pipe<T, N, NSEQ, NT && HAS_NT>);
      (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      int dev = 0, cus = 0, per = 0;
      if (hipGetDevice(&dev) == hipSuccess &&
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
          hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, THREADS, LDS) == hipSuccess && per > 0)
        r = cus * per;
      (void)hipGetLastError();
    });
    return r;
  }

  static int run(GenPipeArgs<T>& a, hipStream_t st) {
    if (THREADS % 64 != 0 || THREADS > pipe_cap<T, N>() || LDS > 160 * 1024) return ST_UNSUPPORTED;
    // one row of the column decode per tile; pair loads of the y-face rows aligned
    if (a.fs.na % (2 * NSEQ) != 0 || (a.inner & 1)) return ST_UNSUPPORTED;
    if (a.g.lb && ((a.g.bpitch & 1) || (a.g.bplane & 1) || (a.g.bslab & 1))) return ST_UNSUPPORTED;
    if ((double)(TPS + 1) * (double)a.inner * (double)sizeof(T) >= 4294967295.0) return ST_UNSUPPORTED;
    if (a.g.lb && (double)(TPS + 1) * (double)a.g.bpitch * (double)sizeof(T) >= 4294967295.0) return ST_UNSUPPORTED;
    // the coefficient prefetch clamps its column indices into the tables (nva >= 1 entries)
    if (a.fs.nva < 1 || a.inner < 2) return ST_UNSUPPORTED;
    const bool nt = HAS_NT && a.inner % (2 * NSEQ) == 0 &&
                    (double)a.outer * (double)a.inner * (double)(N - 1) * sizeof(T) >= NT_STORE_MIN_BYTES;
    const int res = nt ? resident<true>() : resident<false>();
    if (res <= 0) return ST_UNSUPPORTED;
    a.ntile_inner = (a.inner + 2LL * NSEQ - 1) / (2LL * NSEQ);
    const long long ntiles = a.outer * a.ntile_inner;
    if (ntiles <= 0) return ST_OK;
    // the kernel decodes tiles and columns in 32-bit arithmetic
    if (a.inner >= (1LL << 30) || ntiles >= (1LL << 30) || a.fs.na <= 0) return ST_UNSUPPORTED;
    // the y-face pairs into their sums and differences (in place; the arrays are this
    // pass's input only)
    T* lb = const_cast<T*>(a.g.lb);
    if (lb) TRY_ST(face_pm<T>(lb, a.g.bplane, a.outer > 1 ? a.g.bslab : 0, a.g.bplane, a.outer, st));
    const long long grid = ntiles < res ? ntiles : res;
    if (nt)
      hipLaunchKernelGGL((k_gen_pipe<T, N, NSEQ, HAS_NT>), dim3((unsigned)grid), dim3(THREADS), LDS, st, a);
    else
      hipLaunchKernelGGL((k_gen_pipe<T, N, NSEQ, false>), dim3((unsigned)grid), dim3(THREADS), LDS, st, a);
    AHOC_HIP_TRY(hipGetLastError());
    return ST_OK;
  }
};

}  // namespace

}  // namespace fast

template <typename T>
int dst_pipe_pass(int N, const cx<T>* tw, const T* sn, const T* in, T* out, long long outer, long long inner,
                  const DstScale<T>* fused, const DstFaces<T>* faces, int nseq, hipStream_t st) {
  if (inner <= 1 || (inner & 1)) return ST_UNSUPPORTED;
  // plain passes (mode 0), the forward pass with eigen scaling and face sums (mode 1), or a
  // whole slowest-axis Poisson pass: forward, scaling, inverse (mode 2)
  const bool fc = fused != nullptr;
  if (!fc && faces && faces->mode) return ST_UNSUPPORTED;
  const int mode = !fc ? 0 : (faces && faces->mode == 1 ? 1 : 2);
  // the two-transform pass spills registers: at N = 1024 it is 20 % faster than the
  // one-tile kernel in FP64 and 50 % slower in FP32, which keeps the one-tile kernel
  if (mode == 2 && sizeof(T) == 4) return ST_UNSUPPORTED;
  // one slab must stay below 2^31 elements
  if ((double)(N - 1) * (double)inner >= 2147483647.0) return ST_UNSUPPORTED;
  fast::Args<T> a;
  a.in = in;
  a.out = out;
  a.tw = tw;
  a.sn = sn;
  a.outer = outer;
  a.inner = inner;
  a.pitch = inner;
  if (fc) a.fs = *fused;
  if (faces) a.fc = *faces;
#define AHOC_PIPE(NN)                                                                       \
  case NN:                                                                                  \
    return mode == 1 ? fast::PipeLaunch<T, NN, 1>::run(a, nseq, st)                        \
                     : (mode == 2 ? fast::PipeLaunch<T, NN, 2>::run(a, nseq, st)             \
                                  : fast::PipeLaunch<T, NN, 0>::run(a, nseq, st))
  switch (N) {
    AHOC_PIPE(32);
    AHOC_PIPE(64);
    AHOC_PIPE(96);
    AHOC_PIPE(128);
    AHOC_PIPE(192);
    AHOC_PIPE(256);
    AHOC_PIPE(384);
    AHOC_PIPE(512);
    AHOC_PIPE(768);
    AHOC_PIPE(1024);
    AHOC_PIPE(2048);
    AHOC_PIPE(4096);
    default: return ST_UNSUPPORTED;
  }
#undef AHOC_PIPE
}

template <typename T>
int dst_gen_pipe_pass(const DstTables<T>& tb, T* out, long long outer, long long inner, const DstScale<T>& sc,
                      const DstGen<T>& gen, hipStream_t st) {
  if ((double)(tb.N - 1) * (double)inner >= 2147483647.0) return ST_UNSUPPORTED;
  fast::GenPipeArgs<T> a;
  a.out = out;
  a.tw = tb.tw;
  a.sn = tb.sn;
  a.outer = outer;
  a.inner = inner;
  a.ntile_inner = 0;
  a.fs = sc;
  a.g = gen;
  switch (tb.N) {
    case 32: return fast::GenPipeLaunch<T, 32>::run(a, st);
    case 64: return fast::GenPipeLaunch<T, 64>::run(a, st);
    case 96: return fast::GenPipeLaunch<T, 96>::run(a, st);
    case 128: return fast::GenPipeLaunch<T, 128>::run(a, st);
    case 192: return fast::GenPipeLaunch<T, 192>::run(a, st);
    case 256: return fast::GenPipeLaunch<T, 256>::run(a, st);
    case 384: return fast::GenPipeLaunch<T, 384>::run(a, st);
    case 512: return fast::GenPipeLaunch<T, 512>::run(a, st);
    case 768: return fast::GenPipeLaunch<T, 768>::run(a, st);
    case 1024: return fast::GenPipeLaunch<T, 1024>::run(a, st);
    case 2048: return fast::GenPipeLaunch<T, 2048>::run(a, st);
    case 4096: return fast::GenPipeLaunch<T, 4096>::run(a, st);
    default: return ST_UNSUPPORTED;
  }
}

namespace fast {
namespace {

// Launch conditions of the U-solve pass with spectral M (k_dst_pipe MODE 3)
template <typename T, int N> int mpass_check(long long inner, long long na, const DstGen<T>& g) {
  using PLc = PipeLaunch<T, N, 3>;
  if (inner <= 1 || (inner & 1)) return ST_UNSUPPORTED;
  if ((double)(N - 1) * (double)inner >= 2147483647.0) return ST_UNSUPPORTED;
  if (PLc::THREADS % 64 != 0 || PLc::THREADS > pipe_cap<T, N>() || PLc::LDS > 160 * 1024) return ST_UNSUPPORTED;
  if ((double)(PLc::TPS + 1) * (double)inner * (double)sizeof(T) >= 4294967295.0) return ST_UNSUPPORTED;
  // a tile lies in one row of the column decode (one row of the face spectra normal to the
  // fastest axis); the y-face values of a pair are read as one aligned vector
  if (na <= 0 || na % (2 * PLc::NSEQ) != 0) return ST_UNSUPPORTED;
  if (!g.lp || !g.la || !g.wp || !g.wa || !g.ptab) return ST_UNSUPPORTED;
  // y-face spectra [side][column][position] with row pitch bpitch >= N - 1 (byte offsets
  // within one face plane fit 32 bits)
  if (g.lb && (!g.wb || g.bpitch < N - 1 || (double)g.bplane * sizeof(T) >= 4294967295.0)) return ST_UNSUPPORTED;
  if (PLc::template resident<false>() <= 0 || PLc::template resident<true>() <= 0) return ST_UNSUPPORTED;
  return ST_OK;
}

template <typename T, int N>
int mpass_run(const cx<T>* tw, const T* sn, T* buf, long long outer, long long inner, const DstScale<T>& sc,
              const DstFaces<T>& faces, const DstGen<T>& gen, hipStream_t st) {
  TRY_ST((mpass_check<T, N>(inner, sc.na, gen)));
  T* lb = const_cast<T*>(gen.lb);
  if (lb) TRY_ST(face_pm<T>(lb, gen.bplane, outer > 1 ? gen.bslab : 0, gen.bplane, outer, st));
  Args<T> a;
  a.in = buf;
  a.out = buf;
  a.tw = tw;
  a.sn = sn;
  a.outer = outer;
  a.inner = inner;
  a.pitch = inner;
  a.fs = sc;
  a.fc = faces;
  a.fc.mode = 1;
  a.gn = gen;
  return PipeLaunch<T, N, 3>::run(a, 0, st);
}

}  // namespace
}  // namespace fast

#define AHOC_MPASS_CASES(X) X(32) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024) X(2048) X(4096)

template <typename T> bool dst_pipe_mpass_ok(int N, long long inner, long long na, const DstGen<T>& gen) {
  switch (N) {
#define AHOC_MCHK(NN) \
  case NN: return fast::mpass_check<T, NN>(inner, na, gen) == ST_OK;
    AHOC_MPASS_CASES(AHOC_MCHK)
#undef AHOC_MCHK
    default: return false;
  }
}

template <typename T>
int dst_pipe_mpass(int N, const cx<T>* tw, const T* sn, T* buf, long long outer, long long inner,
                   const DstScale<T>& sc, const DstFaces<T>& faces, const DstGen<T>& gen, hipStream_t st) {
  switch (N) {
#define AHOC_MRUN(NN) \
  case NN: return fast::mpass_run<T, NN>(tw, sn, buf, outer, inner, sc, faces, gen, st);
    AHOC_MPASS_CASES(AHOC_MRUN)
#undef AHOC_MRUN
    default: return ST_UNSUPPORTED;
  }
}
#undef AHOC_MPASS_CASES

template bool dst_pipe_mpass_ok<float>(int, long long, long long, const DstGen<float>&);
template bool dst_pipe_mpass_ok<double>(int, long long, long long, const DstGen<double>&);
template int dst_pipe_mpass<float>(int, const cx<float>*, const float*, float*, long long, long long,
                                   const DstScale<float>&, const DstFaces<float>&, const DstGen<float>&, hipStream_t);
template int dst_pipe_mpass<double>(int, const cx<double>*, const double*, double*, long long, long long,
                                    const DstScale<double>&, const DstFaces<double>&, const DstGen<double>&,
                                    hipStream_t);

template int dst_pipe_pass<float>(int, const cx<float>*, const float*, const float*, float*, long long, long long,
                                  const DstScale<float>*, const DstFaces<float>*, int, hipStream_t);
template int dst_pipe_pass<double>(int, const cx<double>*, const double*, const double*, double*, long long,
                                   long long, const DstScale<double>*, const DstFaces<double>*, int, hipStream_t);

template int dst_gen_pipe_pass<float>(const DstTables<float>&, float*, long long, long long,
                                      const DstScale<float>&, const DstGen<float>&, hipStream_t);
template int dst_gen_pipe_pass<double>(const DstTables<double>&, double*, long long, long long,
                                       const DstScale<double>&, const DstGen<double>&, hipStream_t);

}  // namespace ahoc
