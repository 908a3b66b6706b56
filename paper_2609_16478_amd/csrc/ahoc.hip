// Host orchestration and C ABI of the augmented HOC solver (gfx950).
//
// Algorithm 1 of the paper, organised for one GPU:
//   ConstructSchurRHS   b = -R(0): v-solve with Q = 0, u-solve, boundary gather
//   SchurMatVec         homogeneous form R(Q) - R(0) (Lemma 1): lift Q, DST Poisson
//                       solve for V, M(V/alpha), DST Poisson solve for U, gather
//   GMRES(m)            device-resident FP64 Krylov basis, CGS2 Arnoldi, Givens
//   recovery            V from Q^m, then U from V
// Every step runs in HIP kernels; the host only sequences launches and reads
// one scalar per GMRES iteration.  In mixed precision the whole scheme above
// runs in FP32 as the inner solver of an FP64 iterative refinement on the
// coupled system (FP64 residual, FP64 Krylov vectors, FP64 updates).
#include "../../include/ahoc.h"
#include "common.h"
#include "kernels.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <map>
#include <type_traits>
#include <utility>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace ahoc {

static thread_local std::string g_err;
void set_last_error(const char* what, const char* where) {
  g_err = std::string(where ? where : "") + ": " + (what ? what : "");
}

namespace {

template <typename T> struct Prec {
  DstTables<T> tb[3];
  int tile[3] = {0, 0, 0};
  T* s[3] = {nullptr, nullptr, nullptr};
  T* ia = nullptr;    // nodal 1/alpha
  T* af = nullptr;    // alpha on face nodes (N_q)
  T* bufA = nullptr;  // interior work (V)
  T* bufB = nullptr;  // interior work (U)
  T* qT = nullptr;    // N_q, Q in this precision
  T* zq = nullptr;    // N_q zeros
  T* wf[3] = {nullptr, nullptr, nullptr};  // per axis: one-sided face weights w_lo(k), w_hi(k)
  T* wl[3] = {nullptr, nullptr, nullptr};  // per axis: layer sines sin(pi k/N), (-1)^(k+1) sin(pi k/N)
  // face arrays (lift layers / face sums): 3-D x faces [2][n_y'][n_z'], y faces [2][n_z'][px],
  // z faces [2][n_y'][px]; 2-D x faces [2][n_y'], y faces [2][px]
  T* Fx = nullptr;
  T* Fy = nullptr;
  T* Fz = nullptr;
  // spectral entry/exit of the matvec (when every axis has a specialised kernel)
  bool spectral = false;
  // 3-D spectral matvec with the weighting operator M in spectral form: the U-solve's face
  // layers m1 Q_b / alpha_b (layouts as Fx, Fy, Fz) and the scale with the symbol of M
  bool mspec = false;
  T* ptab = nullptr;  // per z position: s_z, layer sine, face weights low/high
  T* Ux = nullptr;
  T* Uy = nullptr;
  T* Uz = nullptr;
  T* mq = nullptr;  // 3-D: m1 / alpha at the boundary node of each face node (Q layout)
  DstScale<T> scM;

  DstScale<T> scV, scU, scP;
  bool ready = false;
};

}  // namespace
}  // namespace ahoc

using namespace ahoc;

struct ahoc_handle {
  ahoc::DevAlloc al;   // device memory provider (the caller's allocator or hipMalloc)
  // recorded on the call's stream after the work of every asynchronous entry point, so
  // ahoc_destroy waits for the handle's own work only
  hipEvent_t done_ev = nullptr;
  bool done_rec = false;
  Geom g;
  Weights w;
  Weights wv;          // the v-equation's lift weights (normal weight shifted by -c m1)
  // triharmonic extension: src_v, src_u and src_t are the sources of the W-, V- and U-solves
  bool tri = false;
  double* src_t = nullptr;
  double cshift = 0;   // the v-equation's shift c = beta/alpha (constant alpha), 0 for beta = 0
  int navier = 0;      // bit f set: face f (2 axis + side) is a Navier face
  // variable beta: nodal c = beta / alpha, the V-solve by BiCGSTAB preconditioned by the
  // sine-transform solve with the constant shift cshift = (min c + max c) / 2
  bool cvar = false;
  double* cnod = nullptr;
  double* bk[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  double* bdot = nullptr;    // device scalars of the BiCGSTAB dot products
  double* bpart = nullptr;   // their partial sums
  double* bpin = nullptr;    // host-pinned copies
  long long vs_iters = 0;    // BiCGSTAB iterations so far (reported per solve)
  double vs_worst = 0;       // largest final relative residual of a V-solve since the last reset
  ahoc_options opt;
  // FP64 problem data
  double* ia64 = nullptr;
  // FP64 V of the V-solve with Q = 0 (the right-hand side's), kept for the recovery: V(Q) is
  // that plus the homogeneous V-solve from Q (spectral FP64 operator, no triharmonic chain)
  double* V0 = nullptr;
  double* af64 = nullptr;
  double* src_v = nullptr;
  double* src_u = nullptr;  // null when g_D = 0
  double* src_q = nullptr;
  double* gD = nullptr;     // nodal copy, null when g_D = 0
  double* vedge = nullptr;  // nodal alpha*lapgD, null when lapgD = 0
  Prec<double> p64;
  Prec<float> p32;
  // refinement state (mixed)
  double *U64 = nullptr, *V64 = nullptr, *Q64 = nullptr;
  float *ru = nullptr, *rv = nullptr, *rq = nullptr;
  // Krylov
  int m = 30;
  int nb_dot = 2048;  // most work-groups of a dot sweep (each >= 2048 entries)
  double *Vb = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr, *gv = nullptr;
  double *h1 = nullptr, *h2 = nullptr, *nrm = nullptr, *part = nullptr, *y = nullptr;
  double *resid = nullptr, *beta = nullptr, *bvec = nullptr, *dq = nullptr, *rvec = nullptr, *R = nullptr;
  double* zvec = nullptr;    // preconditioned Krylov vector
  // GMRES operator (preconditioner and Schur matvec) captured as a HIP graph per operator
  // precision ([0] FP32, [1] FP64), replayed once per Krylov step from the fixed input gin
  // to the fixed output gout; captured on its second use, eager when capture fails
  hipGraphExec_t opg[2] = {nullptr, nullptr};
  int opg_uses[2] = {0, 0};
  bool opg_failed[2] = {false, false};
  double* gin = nullptr;
  double* gout = nullptr;
  long long graph_steps = 0;  // graph replays so far (reported per solve)
  double* b64 = nullptr;     // mixed, Schur refinement: FP64 right-hand side
  // boundary-symbol preconditioner, applied in FP64 for either precision (its low modes
  // are damped ~N-fold, so FP32 rounding of the face transforms would be amplified):
  // inverse 2x2 block coefficients per face mode (Q layout) and FP64 transform tables
  double* pc = nullptr;
  double* qc = nullptr;
  ahoc::DstTables<double> ptb[3];
  bool ptb_own = false;
  int* act = nullptr;        // per instance: a mask (device; zeroing finished segments)
  int* ist = nullptr;        // GMRES state per instance (device): [act | kk | nit | flag | hcnt]
  double* hist = nullptr;    // last 16 residual estimates per instance (device; FP32 stall rule)
  double* eres = nullptr;    // last residual estimate of each instance while active (device)
  double* bn = nullptr;      // ||b|| per instance (device)
  int* pinned_s = nullptr;   // host-pinned image of [act | kk | nit | flag]
  double* pinned_b = nullptr;  // host-pinned ||b|| for the upload
  double* ubuf = nullptr;    // batch: nodal U of all instances before the copy-out
  double* red = nullptr;     // reduction partials
  double* pinned = nullptr;  // host-pinned scalars (2 per instance, at least 8)
  int* pinned_i = nullptr;   // host-pinned ints (one per instance)
  // batch: device table of per-instance pointers, [7][nb] (five input fields, the outputs u,
  // then the Navier data g_L;  // outputs u), and its host image (kept alive while copies from it may be in flight)
  void** ptab = nullptr;
  std::vector<void*> ptab_host;
  std::vector<void*> allocs;
  size_t dev_bytes = 0;      // device memory held by allocs
  // optional per-kernel-class timing with HIP events on the work stream
  bool prof = false;
  std::vector<hipEvent_t> evpool;
  size_t evused = 0;
  struct Pending { int kind; hipEvent_t a, b; double bytes; };
  std::vector<Pending> pending;
  double kms[AHOC_NKIND] = {0};
  long long kcnt[AHOC_NKIND] = {0};
  double kbytes[AHOC_NKIND] = {0};  // accumulated algorithmic bytes
};

namespace ahoc {
namespace {

int dalloc(ahoc_handle* h, void** p, size_t bytes) {
  if (bytes == 0) bytes = 8;
  TRY_ST(dev_alloc(h->al, p, bytes));
  h->allocs.push_back(*p);
  h->dev_bytes += bytes;
  return ST_OK;
}

// Mark the end of the work an entry point enqueued on `st` (waited for by ahoc_destroy).
int mark_done(ahoc_handle* h, hipStream_t st) {
  if (!h->done_ev) return ST_OK;
  AHOC_HIP_TRY(hipEventRecord(h->done_ev, st));
  h->done_rec = true;
  return ST_OK;
}

hipEvent_t tbegin(ahoc_handle* h, hipStream_t st) {
  if (!h->prof) return nullptr;
  if (h->evused + 2 > h->evpool.size()) {
    for (int i = 0; i < 64; ++i) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      h->evpool.push_back(e);
    }
  }
  hipEvent_t a = h->evpool[h->evused++];
  (void)hipEventRecord(a, st);
  return a;
}

void tend(ahoc_handle* h, int kind, hipEvent_t a, double bytes, hipStream_t st) {
  if (!h->prof || !a) return;
  hipEvent_t b = h->evpool[h->evused++];
  (void)hipEventRecord(b, st);
  h->pending.push_back({kind, a, b, bytes});
}

// Fold event pairs into the per-kind totals (waits for each pair's end event).
void tresolve(ahoc_handle* h) {
  for (auto& p : h->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      h->kms[p.kind] += ms;
      h->kcnt[p.kind] += 1;
      h->kbytes[p.kind] += p.bytes;
    }
  }
  h->pending.clear();
  h->evused = 0;
}

#define TRY(...)                \
  do {                          \
    int rc__ = (__VA_ARGS__);   \
    if (rc__) return rc__;      \
  } while (0)

// sizes of whole-batch arrays (nb instances of the per-instance sizes)
inline long long TQ(const Geom& g) { return (long long)g.nb * g.nq; }
inline long long TA(const Geom& g) { return (long long)g.nb * g.nalloc; }
inline long long TN(const Geom& g) { return (long long)g.nb * g.nnodal; }

template <typename T> int alloc_t(ahoc_handle* h, T** p, long long n) {
  return dalloc(h, reinterpret_cast<void**>(p), sizeof(T) * (size_t)n);
}

// interior array (padded rows), zero-filled so the padding columns stay zero
template <typename T> int alloc_int(ahoc_handle* h, T** p, hipStream_t st) {
  int rc = alloc_t(h, p, TA(h->g));
  if (rc) return rc;
  AHOC_HIP_TRY(hipMemsetAsync(*p, 0, sizeof(T) * (size_t)TA(h->g), st));
  return ST_OK;
}

void make_geom(const ahoc_problem* pb, Geom& g) {
  std::memset(&g, 0, sizeof(g));
  g.nb = 1;
  g.dim = pb->dim;
  for (int a = 0; a < 3; ++a) {
    if (a < g.dim) {
      g.n[a] = pb->n[a];
      g.ni[a] = pb->n[a] - 1;
      g.nn[a] = pb->n[a] + 1;
      g.h[a] = (pb->hi[a] - pb->lo[a]) / pb->n[a];
    } else {
      g.n[a] = 2;
      g.ni[a] = 1;
      g.nn[a] = 1;
      g.h[a] = 1.0;
    }
  }
  g.nint = (long long)g.ni[0] * g.ni[1] * g.ni[2];
  g.nnodal = (long long)g.nn[0] * g.nn[1] * g.nn[2];
  // interior rows padded to 32 elements: 128 B aligned rows and column segments
  g.px = ((g.ni[0] + 31) / 32) * 32;
  g.nalloc = (long long)g.px * g.ni[1] * g.ni[2];
  int off = 0;
  for (int a = 0; a < g.dim; ++a) {
    long long fs = 1;
    for (int b = 0; b < g.dim; ++b)
      if (b != a) fs *= g.ni[b];
    g.face_off[2 * a] = off;
    off += (int)fs;
    g.face_off[2 * a + 1] = off;
    off += (int)fs;
  }
  for (int f = 2 * g.dim; f < 7; ++f) g.face_off[f] = off;
  g.nq = off;
}

void make_weights(const Geom& g, Weights& w) {
  const double ix2 = 1.0 / (g.h[0] * g.h[0]), iy2 = 1.0 / (g.h[1] * g.h[1]);
  if (g.dim == 2) {
    // nine-point compact Laplacian
    w.c0 = -20.0 * (ix2 + iy2) / 12.0;
    w.cf[0] = (10.0 * ix2 - 2.0 * iy2) / 12.0;
    w.cf[1] = (10.0 * iy2 - 2.0 * ix2) / 12.0;
    w.cf[2] = 0.0;
    w.ce[0] = (ix2 + iy2) / 12.0;
    w.ce[1] = w.ce[2] = 0.0;
    w.m0 = 8.0 / 12.0;
  } else {
    // 19-point compact Laplacian, planes L_{k-1}, L_k, L_{k+1} with prefactor 1/12
    const double iz2 = 1.0 / (g.h[2] * g.h[2]);
    w.c0 = -16.0 * (ix2 + iy2 + iz2) / 12.0;
    w.cf[0] = (8.0 * ix2 - 2.0 * iy2 - 2.0 * iz2) / 12.0;
    w.cf[1] = (8.0 * iy2 - 2.0 * ix2 - 2.0 * iz2) / 12.0;
    w.cf[2] = (8.0 * iz2 - 2.0 * ix2 - 2.0 * iy2) / 12.0;
    w.ce[0] = (ix2 + iy2) / 12.0;
    w.ce[1] = (ix2 + iz2) / 12.0;
    w.ce[2] = (iy2 + iz2) / 12.0;
    w.m0 = 6.0 / 12.0;
  }
  w.m1 = 1.0 / 12.0;
  w.os[0] = -85.0 / 18.0;
  w.os[1] = 6.0;
  w.os[2] = -1.5;
  w.os[3] = 2.0 / 9.0;
  w.os_gn = 11.0 / 3.0;
}

// Whether every axis has a length-specialised DST kernel (needed for the spectral lift and face sums).
bool faces_available(const Geom& g) {
  if (dst_get_variant() == 1) return false;
  for (int a = 0; a < g.dim; ++a)
    if (!dst_fast_supported(g.n[a])) return false;
  return true;
}

template <typename T> int prec_init(ahoc_handle* h, Prec<T>& P, int tile_opt, hipStream_t st) {
  const Geom& g = h->g;
  for (int a = 0; a < g.dim; ++a) {
    TRY(dst_tables_init<T>(P.tb[a], g.n[a], st, &h->al));
    P.tile[a] = tile_opt > 0 ? tile_opt : 0;  // 0: each kernel picks its default tile
    // eigenvalues of the 1-D second difference on sine mode k: -(4/h^2) sin^2(k pi / (2N))
    std::vector<T> s(g.ni[a]);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int k = 1; k <= g.ni[a]; ++k) {
      const long double sv = sinl(pi * k / (2.0L * g.n[a]));
      s[k - 1] = (T)(-4.0L * sv * sv / ((long double)g.h[a] * g.h[a]));
    }
    TRY(alloc_t(h, &P.s[a], g.ni[a]));
    AHOC_HIP_TRY(hipMemcpyAsync(P.s[a], s.data(), sizeof(T) * g.ni[a], hipMemcpyHostToDevice, st));
    AHOC_HIP_TRY(hipStreamSynchronize(st));
    // 6 U_1 - 3/2 U_2 + 2/9 U_3 of a sine mode k, for the low face (nodes 1,2,3) and the
    // high face (nodes N-1, N-2, N-3, where sin(pi k (N-m)/N) = (-1)^(k+1) sin(pi k m/N))
    std::vector<T> wv(2 * g.ni[a]);
    for (int k = 1; k <= g.ni[a]; ++k) {
      long double acc = 0;
      for (int m = 1; m <= 3; ++m) acc += (long double)h->w.os[m] * sinl(pi * k * m / (long double)g.n[a]);
      wv[k - 1] = (T)acc;
      wv[g.ni[a] + k - 1] = (T)((k % 2 == 1) ? acc : -acc);
    }
    TRY(alloc_t(h, &P.wf[a], 2 * g.ni[a]));
    AHOC_HIP_TRY(hipMemcpyAsync(P.wf[a], wv.data(), sizeof(T) * 2 * g.ni[a], hipMemcpyHostToDevice, st));
    AHOC_HIP_TRY(hipStreamSynchronize(st));
    // sine of mode k at the interior layer next to the low face (node 1) and the high face
    // (node N-1): the normal factor of a face layer's spectrum
    for (int k = 1; k <= g.ni[a]; ++k) {
      const long double sv = sinl(pi * k / (long double)g.n[a]);
      wv[k - 1] = (T)sv;
      wv[g.ni[a] + k - 1] = (T)((k % 2 == 1) ? sv : -sv);
    }
    TRY(alloc_t(h, &P.wl[a], 2 * g.ni[a]));
    AHOC_HIP_TRY(hipMemcpyAsync(P.wl[a], wv.data(), sizeof(T) * 2 * g.ni[a], hipMemcpyHostToDevice, st));
    AHOC_HIP_TRY(hipStreamSynchronize(st));
  }
  if (g.dim == 3) {
    TRY(alloc_t(h, &P.Fx, 2LL * g.ni[1] * g.ni[2]));
    TRY(alloc_t(h, &P.Fy, 2LL * g.px * g.ni[2]));
    TRY(alloc_t(h, &P.Fz, 2LL * g.px * g.ni[1]));
    AHOC_HIP_TRY(hipMemsetAsync(P.Fy, 0, sizeof(T) * 2 * g.px * g.ni[2], st));
    AHOC_HIP_TRY(hipMemsetAsync(P.Fz, 0, sizeof(T) * 2 * g.px * g.ni[1], st));
  } else {  // per instance [2][n_y'] and [2][px]
    TRY(alloc_t(h, &P.Fx, 2LL * g.nb * g.ni[1]));
    TRY(alloc_t(h, &P.Fy, 2LL * g.nb * g.px));
    AHOC_HIP_TRY(hipMemsetAsync(P.Fy, 0, sizeof(T) * 2 * g.nb * g.px, st));
  }
  P.spectral = faces_available(g);
  if (P.spectral && !h->tri) {
    const int t = g.dim - 1;  // the slowest axis
    if (g.dim == 3) {
      TRY(alloc_t(h, &P.Ux, 2LL * g.ni[1] * g.ni[2]));
      TRY(alloc_t(h, &P.Uy, 2LL * g.ni[0] * g.ni[2]));
      TRY(alloc_t(h, &P.Uz, 2LL * g.px * g.ni[1]));
      if (g.nb == 1) {  // m1 / alpha_b in Q layout, for the tiled face-layer pass
        TRY(alloc_t(h, &P.mq, TQ(g)));
        TRY(nodal_to_q<T>(g, h->w.m1, P.ia, P.mq, st));
      }
    } else {  // per instance [2][n_y'] and [2][px]
      TRY(alloc_t(h, &P.Ux, 2LL * g.nb * g.ni[1]));
      TRY(alloc_t(h, &P.Uy, 2LL * g.nb * g.px));
    }
    // (s, layer sine, face weight low, high) per position of the slowest axis, from the
    // tables above
    const int nt = g.ni[t];
    std::vector<T> hs(nt), hl(2 * nt), hw(2 * nt), pt(4 * (size_t)nt);
    AHOC_HIP_TRY(hipMemcpyAsync(hs.data(), P.s[t], sizeof(T) * nt, hipMemcpyDeviceToHost, st));
    AHOC_HIP_TRY(hipMemcpyAsync(hl.data(), P.wl[t], sizeof(T) * 2 * nt, hipMemcpyDeviceToHost, st));
    AHOC_HIP_TRY(hipMemcpyAsync(hw.data(), P.wf[t], sizeof(T) * 2 * nt, hipMemcpyDeviceToHost, st));
    AHOC_HIP_TRY(hipStreamSynchronize(st));
    for (int k = 0; k < nt; ++k) {
      pt[4 * k] = hs[k];
      pt[4 * k + 1] = hl[k];
      pt[4 * k + 2] = hw[k];
      pt[4 * k + 3] = hw[nt + k];
    }
    TRY(alloc_t(h, &P.ptab, 4LL * nt));
    AHOC_HIP_TRY(hipMemcpyAsync(P.ptab, pt.data(), sizeof(T) * 4 * nt, hipMemcpyHostToDevice, st));
    AHOC_HIP_TRY(hipStreamSynchronize(st));
    const long long inner = g.dim == 3 ? (long long)g.px * g.ni[1] : g.px;
    P.mspec = dst_pipe_mpass_ok<T>(g.n[t], inner, g.px, mspec_gen<T>(g, P));
  }
  TRY(alloc_int(h, &P.bufA, st));
  TRY(alloc_int(h, &P.bufB, st));
  // setup-time choice between the FFT and the matrix-core pass for the plain passes of the
  // operator, timed on their own shapes: the x (row) passes; in 3-D also the strided y passes
  if (g.dim == 2) {
    TRY(dst_autotune<T>(P.tb[0], P.bufA, (long long)g.nb * g.ni[1], 1, g.px, st));
  } else {
    TRY(dst_autotune<T>(P.tb[0], P.bufA, (long long)g.ni[1] * g.ni[2], 1, g.px, st));
    TRY(dst_autotune<T>(P.tb[1], P.bufA, g.ni[2], g.px, g.px, st));
  }
  AHOC_HIP_TRY(hipMemsetAsync(P.bufA, 0, sizeof(T) * (size_t)TA(g), st));
  TRY(alloc_t(h, &P.qT, TQ(g)));
  TRY(alloc_t(h, &P.zq, TQ(g)));
  AHOC_HIP_TRY(hipMemsetAsync(P.zq, 0, sizeof(T) * TQ(g), st));
  double norm = 1.0;
  for (int a = 0; a < g.dim; ++a) norm *= 2.0 / g.n[a];
  const int t = g.dim - 1;
  DstScale<T> sc;
  sc.s_this = P.s[t];
  sc.s_a = P.s[0];
  sc.na = g.px;
  sc.nva = g.ni[0];
  if (g.dim == 3) {
    sc.s_b = P.s[1];
    sc.c_ta = (T)((g.h[2] * g.h[2] + g.h[0] * g.h[0]) / 12.0);
    sc.c_tb = (T)((g.h[2] * g.h[2] + g.h[1] * g.h[1]) / 12.0);
    sc.c_ab = (T)((g.h[0] * g.h[0] + g.h[1] * g.h[1]) / 12.0);
  } else {
    sc.s_b = nullptr;
    sc.c_ta = (T)((g.h[1] * g.h[1] + g.h[0] * g.h[0]) / 12.0);
    sc.c_tb = 0;
    sc.c_ab = 0;
  }
  P.scV = sc;
  P.scV.scale = (T)(-norm);  // V = -L^{-1}(...)
  if (h->cshift != 0.0) {
    // V = -(L - c M)^{-1}(...): lambda_L - c mu_M, mu_M = m0 + 2 m1 sum_a (1 + h_a^2 s_a / 2)
    const double c = h->cshift, m0 = h->w.m0, m1 = h->w.m1;
    P.scV.a0 = (T)(-c * (m0 + 2.0 * m1 * g.dim));
    P.scV.ka = (T)(-c * m1 * g.h[0] * g.h[0]);
    P.scV.kb = g.dim == 3 ? (T)(-c * m1 * g.h[1] * g.h[1]) : (T)0;
    P.scV.kt = (T)(-c * m1 * g.h[t] * g.h[t]);
  }
  P.scU = sc;
  P.scU.scale = (T)norm;     // U = +L^{-1}(...)
  P.scP = P.scU;
  // the U-solve with spectral M: mu_M = m0 + 2 dim m1 + m1 sum_a h_a^2 s_a
  P.scM = P.scU;
  P.scM.mc0 = (T)(h->w.m0 + 2.0 * g.dim * h->w.m1);
  P.scM.mca = (T)(h->w.m1 * g.h[0] * g.h[0]);
  P.scM.mcb = g.dim == 3 ? (T)(h->w.m1 * g.h[1] * g.h[1]) : (T)0;
  P.scM.mct = (T)(h->w.m1 * g.h[t] * g.h[t]);
  P.ready = true;
  return ST_OK;
}

template <typename T> void prec_free(Prec<T>& P) {
  for (int a = 0; a < 3; ++a) dst_tables_free(P.tb[a]);
  P.ready = false;
}

// Dirichlet solve on an interior array: buf <- scale * S (S in / lambda), in place unless
// `in` is given (then the first pass reads it and `in` is left unchanged).
template <typename T>
int poisson(ahoc_handle* h, Prec<T>& P, T* buf, const DstScale<T>& sc, hipStream_t st, const T* in = nullptr,
            const RowLift<T>* lf = nullptr) {
  const Geom& g = h->g;
  const double pass_bytes = 2.0 * (double)g.nint * g.nb * sizeof(T);  // one read + one write of the array
  const T* src = in ? in : buf;
  bool first = true;
  auto run = [&](int kind, const DstTables<T>& tb, long long outer, long long inner,
                 const DstScale<T>* f, int tile) -> int {
    hipEvent_t e = tbegin(h, st);
    // with lf, the first (row) pass adds the lift's face layers to its input while loading
    const int rc = (first && lf) ? dst_rows_lift_pass<T>(tb.N, tb.tw, tb.sn, src, buf, outer, g.px, *lf, st)
                                 : dst_pass<T>(tb, src, buf, outer, inner, g.px, f, tile, st);
    first = false;
    src = buf;
    tend(h, kind, e, pass_bytes, st);
    return rc;
  };
  // strided passes also transform the (zero) padding columns of each row
  if (g.dim == 2) {  // a batch: nb slabs of n_y' rows
    TRY(run(AHOC_K_DST_ROWS, P.tb[0], (long long)g.nb * g.ni[1], 1, nullptr, P.tile[0]));
    TRY(run(AHOC_K_DST_FUSED, P.tb[1], g.nb, g.px, &sc, P.tile[1]));
    TRY(run(AHOC_K_DST_ROWS, P.tb[0], (long long)g.nb * g.ni[1], 1, nullptr, P.tile[0]));
  } else {
    const long long rows = (long long)g.ni[1] * g.ni[2];
    TRY(run(AHOC_K_DST_ROWS, P.tb[0], rows, 1, nullptr, P.tile[0]));
    TRY(run(AHOC_K_DST_STRIDED, P.tb[1], g.ni[2], g.px, nullptr, P.tile[1]));
    TRY(run(AHOC_K_DST_FUSED, P.tb[2], 1, (long long)g.px * g.ni[1], &sc, P.tile[2]));
    TRY(run(AHOC_K_DST_STRIDED, P.tb[1], g.ni[2], g.px, nullptr, P.tile[1]));
    TRY(run(AHOC_K_DST_ROWS, P.tb[0], rows, 1, nullptr, P.tile[0]));
  }
  return ST_OK;
}

// Variable beta (Remark 2): the interior V of -L_h V + M(c V) = src with V = Q on the face
// interiors, c = beta / alpha nodal, into P.bufA.  BiCGSTAB on A x = src - A_IB Q (A the
// interior operator), right-preconditioned by K = -L_h + cshift M, whose inverse is one
// sine-transform solve.  Stops at ||r|| <= 1e-14 ||rhs|| (the FP64 rounding level of the
// preconditioned operator), after vsolve_max_iters (200) iterations, when four iterations
// gained less than a factor 2, or on a breakdown (a zero or non-finite rho or step),
// keeping the last iterate.  The final ||r|| / ||rhs|| of every V-solve is folded into
// h->vs_worst, which the solve reports and checks against VSOLVE_RELRES_MAX.
constexpr int VS_DOT_BLOCKS = 2048;  // work-groups of the V-solve's dot sweeps (>= 2048 entries each)

int vsolve_var(ahoc_handle* h, Prec<double>& P, const double* Q, const double* src, hipStream_t st) {
  const Geom& g = h->g;
  const long long n = TA(g);
  // rh, r, t are consecutive n-vectors so that <rh, r>, <r, r> and <r, t>, <t, t> are one
  // two-vector sweep each
  double *x = P.bufA, *rh = h->bk[0], *r = h->bk[1], *t = h->bk[2], *p = h->bk[3], *v = h->bk[4],
         *y = h->bk[5], *z = h->bk[6];
  const int nbk = (int)std::max<long long>(1, std::min<long long>(VS_DOT_BLOCKS, n / 2048));
  // <V_j, w> for the nv consecutive vectors V_0.. (n apart) into bpin[0..nv) (synchronising)
  auto dots = [&](const double* V, int nv, const double* w) -> int {
    TRY(mdot_partial(V, n, nv, w, n, 1, h->bpart, nbk, st));
    TRY(mdot_reduce(h->bpart, nbk, nv, 1, h->bdot, nv, 0, st));
    AHOC_HIP_TRY(hipMemcpyAsync(h->bpin, h->bdot, sizeof(double) * nv, hipMemcpyDeviceToHost, st));
    AHOC_HIP_TRY(hipStreamSynchronize(st));
    return ST_OK;
  };
  // y += a x and the reduced <u, y>, <y, y> into bpin[0], bpin[1] (synchronising)
  auto update_dots = [&](double a, const double* xv, double* yv, const double* u) -> int {
    TRY(axpy_dot2(n, a, xv, yv, u, h->bpart, nbk, st));
    TRY(mdot_reduce(h->bpart, nbk, 2, 1, h->bdot, 2, 0, st));
    AHOC_HIP_TRY(hipMemcpyAsync(h->bpin, h->bdot, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
    AHOC_HIP_TRY(hipStreamSynchronize(st));
    return ST_OK;
  };
  auto apply = [&](const double* in, double* out) { return vapply(g, h->w, in, nullptr, h->cnod, nullptr, out, st); };
  auto precond = [&](const double* in, double* out) { return poisson<double>(h, P, out, P.scV, st, in); };
  hipEvent_t e = tbegin(h, st);
  // r = src - A_IB Q  (x = 0)
  TRY(fill(n, 0.0, x, st));
  TRY(vapply(g, h->w, x, Q, h->cnod, src, r, st));
  TRY(axpby(n, 0.0, r, -1.0, r, st));
  AHOC_HIP_TRY(hipMemcpyAsync(rh, r, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  TRY(dots(rh, 2, r));  // <rh, r> = <r, r>
  const double bnorm = std::sqrt(h->bpin[1]);
  if (bnorm == 0.0) {
    tend(h, AHOC_K_VSOLVE, e, 0.0, st);
    return ST_OK;
  }
  TRY(fill(n, 0.0, p, st));
  TRY(fill(n, 0.0, v, st));
  double rho = 1.0, alpha = 1.0, omega = 1.0, best = bnorm, rho1 = h->bpin[0];
  double last = bnorm;  // ||r|| of the current iterate
  int since = 0;
  const int cap = h->opt.vsolve_max_iters > 0 ? h->opt.vsolve_max_iters : 200;
  for (int it = 0; it < cap; ++it) {
    if (rho1 == 0.0 || !std::isfinite(rho1)) break;
    const double beta = (rho1 / rho) * (alpha / omega);
    TRY(lin3(n, 1.0, r, -beta * omega, v, beta, p, st));  // p = r + beta (p - omega v)
    TRY(precond(p, y));
    TRY(apply(y, v));
    TRY(dots(v, 1, rh));
    if (h->bpin[0] == 0.0 || !std::isfinite(h->bpin[0])) break;
    alpha = rho1 / h->bpin[0];
    TRY(update_dots(-alpha, v, r, nullptr));  // s = r - alpha v, in r; <s, s>
    ++h->vs_iters;
    double rn = std::sqrt(h->bpin[1]);
    if (rn <= 1e-14 * bnorm) {
      TRY(axpby(n, alpha, y, 1.0, x, st));  // x += alpha y
      last = rn;
      break;
    }
    TRY(precond(r, z));
    TRY(apply(z, t));
    TRY(dots(r, 2, t));  // <s, t>, <t, t>
    if (h->bpin[1] == 0.0 || !std::isfinite(h->bpin[0] / h->bpin[1])) {
      TRY(axpby(n, alpha, y, 1.0, x, st));  // keep the half step
      last = rn;
      break;
    }
    omega = h->bpin[0] / h->bpin[1];
    TRY(lin3(n, alpha, y, omega, z, 1.0, x, st));  // x += alpha y + omega z
    TRY(update_dots(-omega, t, r, rh));  // r = s - omega t; <rh, r> for the next step, <r, r>
    rn = std::sqrt(h->bpin[1]);
    last = rn;
    rho = rho1;
    rho1 = h->bpin[0];
    if (rn <= 1e-14 * bnorm) break;
    if (rn < 0.5 * best) {
      best = rn;
      since = 0;
    } else if (++since >= 4) {
      break;
    }
  }
  const double rel = std::isfinite(last) ? last / bnorm : HUGE_VAL;
  h->vs_worst = std::max(h->vs_worst, rel);
  tend(h, AHOC_K_VSOLVE, e, 0.0, st);
  return ST_OK;
}

// V-solves whose final relative residual exceeds this leave the Schur operator inexact:
// the solve then reports AHOC_E_NOCONV.
constexpr double VSOLVE_RELRES_MAX = 1e-10;

// V = -L^{-1}(src + L_bnd[Q])  into P.bufA
template <typename T> int vsolve(ahoc_handle* h, Prec<T>& P, const T* Q, const T* src, hipStream_t st) {
  if (h->cvar) {
    if constexpr (std::is_same<T, double>::value) return vsolve_var(h, P, Q, src, st);
    else return ST_UNSUPPORTED;
  }
  const Geom& g = h->g;
  hipEvent_t e = tbegin(h, st);
  const long long rows = g.dim == 3 ? (long long)g.ni[1] * g.ni[2] : (long long)g.nb * g.ni[1];
  if (src && P.spectral && dst_get_variant() != 4 && dst_rows_lift_supported<T>(g.n[0], rows, g.px)) {
    // the lift as face layers (the spectral path's kernel), added to the source by the
    // Poisson solve's first row pass while it loads: no lift pass over the volume
    TRY(face_lift<T>(g, h->wv, Q, P.Fx, P.Fy, P.Fz, st));
    tend(h, AHOC_K_LIFT, e, (double)TQ(g) * 2.0 * sizeof(T), st);
    RowLift<T> lf;
    lf.dim = g.dim;
    lf.ni1 = g.ni[1];
    lf.ni2 = g.dim == 3 ? g.ni[2] : 1;
    lf.px = g.px;
    lf.lx = P.Fx;
    lf.ly = P.Fy;
    lf.lz = g.dim == 3 ? P.Fz : nullptr;
    lf.xplane = g.dim == 3 ? (long long)g.ni[1] * g.ni[2] : g.ni[1];
    lf.yplane = g.dim == 3 ? (long long)g.ni[2] * g.px : g.px;
    lf.zplane = g.dim == 3 ? (long long)g.ni[1] * g.px : 0;
    return poisson<T>(h, P, P.bufA, P.scV, st, src, &lf);
  }
  TRY(lift<T>(g, h->wv, Q, src, P.bufA, st));
  tend(h, AHOC_K_LIFT, e, (double)g.nint * g.nb * sizeof(T) * (src ? 2 : 1), st);
  return poisson<T>(h, P, P.bufA, P.scV, st);
}

// U = L^{-1}(M(V/alpha) + src)  with V = P.bufA, into P.bufB
template <typename T> int usolve(ahoc_handle* h, Prec<T>& P, const T* Q, const T* src, hipStream_t st) {
  hipEvent_t e = tbegin(h, st);
  TRY(rhs_u<T>(h->g, h->w, P.bufA, Q, P.ia, src, P.bufB, st));
  // reads V and 1/alpha (nodal), writes G
  tend(h, AHOC_K_RHS_U, e, h->g.nb * ((double)sizeof(T) * (2.0 * h->g.nint + h->g.nnodal) + (src ? h->g.nint * sizeof(T) : 0)), st);
  return poisson<T>(h, P, P.bufB, P.scU, st);
}

// 2-D DST-I of every face array, in place (the unnormalised transform is its own inverse
// up to the factor folded into the eigen scaling).
template <typename T> int face_dst2(ahoc_handle* h, Prec<T>& P, T* Fx, T* Fy, T* Fz, hipStream_t st) {
  const Geom& g = h->g;
  if (g.dim == 3) {
    TRY(dst_pass<T>(P.tb[0], Fz, Fz, 2LL * g.ni[1], 1, g.px, nullptr, 0, st));
    TRY(dst_pass<T>(P.tb[1], Fz, Fz, 2, g.px, g.px, nullptr, 0, st));
    TRY(dst_pass<T>(P.tb[2], Fx, Fx, 2LL * g.ni[1], 1, g.ni[2], nullptr, 0, st));
    TRY(dst_pass<T>(P.tb[1], Fx, Fx, 2, g.ni[2], g.ni[2], nullptr, 0, st));
    TRY(dst_pass<T>(P.tb[0], Fy, Fy, 2LL * g.ni[2], 1, g.px, nullptr, 0, st));
    TRY(dst_pass<T>(P.tb[2], Fy, Fy, 2, g.px, g.px, nullptr, 0, st));
  } else {
    TRY(dst_pass<T>(P.tb[0], Fy, Fy, 2LL * g.nb, 1, g.px, nullptr, 0, st));
    TRY(dst_pass<T>(P.tb[1], Fx, Fx, 2LL * g.nb, 1, g.ni[1], nullptr, 0, st));
  }
  return ST_OK;
}
template <typename T> int face_dst2(ahoc_handle* h, Prec<T>& P, hipStream_t st) {
  return face_dst2<T>(h, P, P.Fx, P.Fy, P.Fz, st);
}

// Homogeneous V-solve V = -L^{-1} L_h^bnd[Q] into P.bufA through the spectral lift: face
// layers of the lift, their 2-D spectra, then the slowest-axis pass generates the 3-D
// spectrum, scales it and inverts along its axis; the other axes are inverted as usual.
template <typename T>
int vsolve_spec(ahoc_handle* h, Prec<T>& P, const T* Q, hipStream_t st, bool skip_x = false, bool lifted = false,
                const T* addv = nullptr) {
  const Geom& g = h->g;
  if (!lifted) {  // (else the face layers are in Fx, Fy, Fz already)
    hipEvent_t e = tbegin(h, st);
    TRY(face_lift<T>(g, h->wv, Q, P.Fx, P.Fy, P.Fz, st));
    TRY(face_dst2<T>(h, P, st));
    tend(h, AHOC_K_LIFT, e, (double)TQ(g) * 2.0 * sizeof(T), st);
  }
  const double pass_bytes = 2.0 * (double)g.nint * g.nb * sizeof(T);
  T* buf = P.bufA;
  DstGen<T> gen;
  gen.wa = P.wl[0];
  gen.nwa = g.ni[0];
  gen.la = P.Fx;
  hipEvent_t eg = tbegin(h, st);
  if (g.dim == 3) {
    gen.lp = P.Fz;
    gen.pplane = (long long)g.px * g.ni[1];
    gen.wp = P.wl[2];
    gen.aplane = (long long)g.ni[1] * g.ni[2];
    gen.apitch = 1;
    gen.arow = g.ni[2];
    gen.lb = P.Fy;
    gen.bplane = (long long)g.px * g.ni[2];
    gen.bpitch = g.px;
    gen.wb = P.wl[1];
    gen.nwb = g.ni[1];
    TRY(dst_gen_pass<T>(P.tb[2], buf, 1, (long long)g.px * g.ni[1], P.scV, gen, st));
  } else {
    gen.lp = P.Fy;
    gen.pplane = g.px;
    gen.wp = P.wl[1];
    gen.aplane = g.ni[1];
    gen.apitch = 1;
    gen.pslab = 2LL * g.px;  // instance o of a batch
    gen.aslab = 2LL * g.ni[1];
    TRY(dst_gen_pass<T>(P.tb[1], buf, g.nb, g.px, P.scV, gen, st));
  }
  tend(h, AHOC_K_DST_GEN, eg, (double)g.nint * g.nb * sizeof(T), st);
  auto run = [&](int kind, const DstTables<T>& tb, long long outer, long long inner, int tile) -> int {
    hipEvent_t ev = tbegin(h, st);
    const int rc = dst_pass<T>(tb, buf, buf, outer, inner, g.px, nullptr, tile, st);
    tend(h, kind, ev, pass_bytes, st);
    return rc;
  };
  if (g.dim == 3) TRY(run(AHOC_K_DST_STRIDED, P.tb[1], g.ni[2], g.px, P.tile[1]));
  if (!skip_x) {
    const long long rows = g.dim == 3 ? (long long)g.ni[1] * g.ni[2] : (long long)g.nb * g.ni[1];
    if (addv) {
      // V = addv + this solve: the addend enters the last row pass (FFT row kernel) or,
      // where that kernel does not run, an axpy after the chosen pass
      int rc = ST_UNSUPPORTED;
      if (dst_get_variant() == 0 || dst_get_variant() == 5) {
        hipEvent_t ev = tbegin(h, st);
        rc = dst_rows_add_pass<T>(g.n[0], P.tb[0].tw, P.tb[0].sn, buf, buf, addv, rows, g.px, st);
        tend(h, AHOC_K_DST_ROWS, ev, pass_bytes * 1.5, st);
      }
      if (rc == ST_UNSUPPORTED) {
        TRY(run(AHOC_K_DST_ROWS, P.tb[0], rows, 1, P.tile[0]));
        if constexpr (std::is_same<T, double>::value) TRY(axpby(TA(g), 1.0, addv, 1.0, buf, st));
        else return ST_UNSUPPORTED;
      } else {
        TRY(rc);
      }
    } else {
      TRY(run(AHOC_K_DST_ROWS, P.tb[0], rows, 1, P.tile[0]));
    }
  }
  return ST_OK;
}

// Face-array arguments of the U-solve pass with spectral M (layouts as the V-solve's lift)
template <typename T> DstGen<T> mspec_gen(const Geom& g, Prec<T>& P) {
  DstGen<T> gen;
  gen.wa = P.wl[0];
  gen.nwa = g.ni[0];
  gen.la = P.Ux;
  gen.apitch = 1;
  gen.ptab = P.ptab;
  if (g.dim == 3) {
    gen.lp = P.Uz;
    gen.pplane = (long long)g.px * g.ni[1];
    gen.wp = P.wl[2];
    gen.aplane = (long long)g.ni[1] * g.ni[2];
    gen.arow = g.ni[2];
    gen.lb = P.Uy;  // [side][i][k], k fastest
    gen.bplane = (long long)g.ni[0] * g.ni[2];
    gen.bpitch = g.ni[2];
    gen.wb = P.wl[1];
    gen.nwb = g.ni[1];
  } else {  // instance o of a batch: y faces [o][2][px], x faces [o][2][n_y']
    gen.lp = P.Uy;
    gen.pplane = g.px;
    gen.pslab = 2LL * g.px;
    gen.wp = P.wl[1];
    gen.aplane = g.ni[1];
    gen.aslab = 2LL * g.ni[1];
  }
  return gen;
}

// Homogeneous 3-D Schur matvec with the weighting operator M in spectral form.  M is
// diagonalised by the sine transforms: on the interior values W = V / alpha (zero on the
// boundary) it is the symbol mu_M = m0 + 2 m1 sum_a cos(theta_a), and its coupling of the
// layers next to the faces to the face values W_b = Q_b / alpha_b is a face-layer source
// m1 W_b, whose spectrum is one layer sine times a 2-D face spectrum (as the V-solve's
// lift).  So U = L^-1 M (V / alpha) in spectral form is (mu_M W^ + G^) / lambda_L:
//   V-solve: spectral lift, generated z inverse, y inverse;
//   x: inverse of the V-solve, times 1/alpha, forward of the U-solve (one pass);
//   y forward; z forward with mu_M / lambda_L, the face-layer term and the z-face sums;
//   x/y-face sums of the scaled spectrum; 2-D inverse transforms of the face sums; gather.
// The volume is read and written in place in bufA.
template <typename T> int matvec_mspec(ahoc_handle* h, Prec<T>& P, const T* Q, double* y, hipStream_t st) {
  const Geom& g = h->g;
  const bool d3 = g.dim == 3;
  const bool tiled = d3 && P.mq;
  if (tiled) {
    // both face-layer sets in one pass over Q, then the V-solve's layer spectra
    hipEvent_t e = tbegin(h, st);
    TRY(face_lifts3<T>(g, h->wv, Q, P.mq, P.Fx, P.Fy, P.Fz, P.Ux, P.Uy, P.Uz, st));
    TRY(face_dst2<T>(h, P, st));
    tend(h, AHOC_K_LIFT, e, (double)TQ(g) * 4.0 * sizeof(T), st);
  }
  TRY(vsolve_spec<T>(h, P, Q, st, true, tiled));
  hipEvent_t el = tbegin(h, st);
  if (!tiled) TRY(face_lift_m<T>(g, h->w, Q, P.ia, P.Ux, P.Uy, P.Uz, st));
  if (d3) {
    // 2-D spectra: x and z faces as the lift's; y faces [2][n_x'][n_z'] (z rows, x strided)
    TRY(dst_pass<T>(P.tb[0], P.Uz, P.Uz, 2LL * g.ni[1], 1, g.px, nullptr, 0, st));
    TRY(dst_pass<T>(P.tb[1], P.Uz, P.Uz, 2, g.px, g.px, nullptr, 0, st));
    TRY(dst_pass<T>(P.tb[2], P.Ux, P.Ux, 2LL * g.ni[1], 1, g.ni[2], nullptr, 0, st));
    TRY(dst_pass<T>(P.tb[1], P.Ux, P.Ux, 2, g.ni[2], g.ni[2], nullptr, 0, st));
    TRY(dst_pass<T>(P.tb[2], P.Uy, P.Uy, 2LL * g.ni[0], 1, g.ni[2], nullptr, 0, st));
    TRY(dst_pass<T>(P.tb[0], P.Uy, P.Uy, 2, g.ni[2], g.ni[2], nullptr, 0, st));
  } else {
    TRY(face_dst2<T>(h, P, P.Ux, P.Uy, nullptr, st));
  }
  tend(h, AHOC_K_LIFT, el, (double)TQ(g) * 3.0 * sizeof(T), st);
  T* buf = P.bufA;
  const double vol = (double)g.nint * g.nb * sizeof(T);
  const long long rows = d3 ? (long long)g.ni[1] * g.ni[2] : (long long)g.nb * g.ni[1];
  hipEvent_t ex = tbegin(h, st);
  TRY(dst_rows_mul_pass<T>(g.n[0], P.tb[0].tw, P.tb[0].sn, buf, buf, rows, g.px, P.ia, g.ni[1], d3 ? 1 : 0,
                           g.nn[0], g.nn[1], st));
  tend(h, AHOC_K_DST_XMUL, ex, 2.0 * vol + (double)g.nnodal * g.nb * sizeof(T), st);
  if (d3) {
    hipEvent_t ey = tbegin(h, st);
    TRY(dst_pass<T>(P.tb[1], buf, buf, g.ni[2], g.px, g.px, nullptr, P.tile[1], st));
    tend(h, AHOC_K_DST_STRIDED, ey, 2.0 * vol, st);
  }
  DstFaces<T> fp;
  fp.mode = 1;
  if (d3) {
    fp.out = P.Fz;
    fp.w = P.wf[2];
    fp.plane = (long long)g.px * g.ni[1];
  } else {
    fp.out = P.Fy;
    fp.w = P.wf[1];
    fp.plane = g.px;
    fp.slab = 2LL * g.px;  // instance o of a batch
  }
  const int t = g.dim - 1;
  hipEvent_t ez = tbegin(h, st);
  TRY(dst_pipe_mpass<T>(g.n[t], P.tb[t].tw, P.tb[t].sn, buf, d3 ? 1 : g.nb, d3 ? (long long)g.px * g.ni[1] : g.px,
                        P.scM, fp, mspec_gen<T>(g, P), st));
  tend(h, AHOC_K_DST_FUSED, ez, 2.0 * vol, st);
  hipEvent_t er = tbegin(h, st);
  if (d3)
    TRY(face_reduce<T>(buf, g.ni[2], g.ni[1], g.ni[0], g.px, P.wf[0], P.wf[1], P.Fx, P.Fy,
                       (long long)g.ni[2] * g.ni[1], 1, g.ni[2], st));
  else
    TRY(face_reduce<T>(buf, g.nb, g.ni[1], g.ni[0], g.px, P.wf[0], nullptr, P.Fx, nullptr, g.ni[1],
                       2LL * g.ni[1], 1, st));
  tend(h, AHOC_K_FACE_REDUCE, er, vol, st);
  hipEvent_t ef = tbegin(h, st);
  TRY(face_dst2<T>(h, P, st));
  TRY(gather_faces<T>(g, P.Fx, P.Fy, P.Fz, Q, P.af, nullptr, y, st));
  tend(h, AHOC_K_GATHER, ef, (double)TQ(g) * (5 * sizeof(T) + sizeof(double)), st);
  return ST_OK;
}

// U-solve for the boundary residual only: U = L^{-1}(M(V/alpha) + src) is never formed.
// The forward transforms run as usual; the slowest-axis pass scales the spectrum, forms
// the face sums along its own axis and stores the scaled spectrum; one streaming
// reduction forms the sums along the other two axes, and 2-D inverse transforms of the
// face arrays give the combination 6 U_1 - 3/2 U_2 + 2/9 U_3 next to each face.
template <typename T> int usolve_spec(ahoc_handle* h, Prec<T>& P, const T* Q, const T* src, hipStream_t st) {
  const Geom& g = h->g;
  hipEvent_t e = tbegin(h, st);
  TRY(rhs_u<T>(g, h->w, P.bufA, Q, P.ia, src, P.bufB, st));
  tend(h, AHOC_K_RHS_U, e, g.nb * ((double)sizeof(T) * (2.0 * g.nint + g.nnodal) + (src ? g.nint * sizeof(T) : 0)), st);
  T* buf = P.bufB;
  const double pass_bytes = 2.0 * (double)g.nint * g.nb * sizeof(T);
  auto run = [&](int kind, const DstTables<T>& tb, long long outer, long long inner, const DstScale<T>* f,
                 int tile, const DstFaces<T>* fc) -> int {
    hipEvent_t ev = tbegin(h, st);
    const int rc = dst_pass<T>(tb, buf, buf, outer, inner, g.px, f, tile, st, fc);
    tend(h, kind, ev, pass_bytes, st);
    return rc;
  };
  DstFaces<T> fp;
  fp.mode = 1;
  if (g.dim == 3) {
    fp.out = P.Fz;
    fp.w = P.wf[2];
    fp.plane = (long long)g.px * g.ni[1];
    TRY(run(AHOC_K_DST_ROWS, P.tb[0], (long long)g.ni[1] * g.ni[2], 1, nullptr, P.tile[0], nullptr));
    TRY(run(AHOC_K_DST_STRIDED, P.tb[1], g.ni[2], g.px, nullptr, P.tile[1], nullptr));
    TRY(run(AHOC_K_DST_FUSED, P.tb[2], 1, (long long)g.px * g.ni[1], &P.scU, P.tile[2], &fp));
    hipEvent_t er = tbegin(h, st);
    TRY(face_reduce<T>(buf, g.ni[2], g.ni[1], g.ni[0], g.px, P.wf[0], P.wf[1], P.Fx, P.Fy,
                       (long long)g.ni[2] * g.ni[1], 1, g.ni[2], st));
    tend(h, AHOC_K_FACE_REDUCE, er, (double)g.nint * sizeof(T), st);
  } else {
    fp.out = P.Fy;
    fp.w = P.wf[1];
    fp.plane = g.px;
    fp.slab = 2LL * g.px;  // instance o of a batch
    TRY(run(AHOC_K_DST_ROWS, P.tb[0], (long long)g.nb * g.ni[1], 1, nullptr, P.tile[0], nullptr));
    TRY(run(AHOC_K_DST_FUSED, P.tb[1], g.nb, g.px, &P.scU, P.tile[1], &fp));
    hipEvent_t er = tbegin(h, st);
    TRY(face_reduce<T>(buf, g.nb, g.ni[1], g.ni[0], g.px, P.wf[0], nullptr, P.Fx, nullptr, g.ni[1],
                       2LL * g.ni[1], 1, st));
    tend(h, AHOC_K_FACE_REDUCE, er, (double)g.nint * g.nb * sizeof(T), st);
  }
  hipEvent_t ef = tbegin(h, st);
  TRY(face_dst2<T>(h, P, st));
  tend(h, AHOC_K_GATHER, ef, (double)TQ(g) * 2.0 * sizeof(T), st);
  return ST_OK;
}

// Boundary-symbol preconditioner: FP64 symbol tables, the inverse block coefficients
// and FP64 DST tables for the face transforms (shared with the FP64 operator if any).
int precond_init(ahoc_handle* h, hipStream_t st) {
  const Geom& g = h->g;
  std::vector<double*> tabs(12, nullptr);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int a = 0; a < g.dim; ++a) {
    const int L = g.ni[a];
    std::vector<double> tv(4 * (size_t)L);
    for (int k = 1; k <= L; ++k) {
      const long double sh = sinl(pi * k / (2.0L * g.n[a]));
      tv[k - 1] = (double)(-4.0L * sh * sh / ((long double)g.h[a] * g.h[a]));
      tv[L + k - 1] = (double)cosl(pi * k / (long double)g.n[a]);
      tv[2 * L + k - 1] = (double)sinl(pi * k / (long double)g.n[a]);
      long double acc = 0;
      if (h->tri) {  // the triharmonic q-row's fourth-derivative combination of U_1..U_4
        const long double a4[4] = {-104.0L, 57.0L / 2.0L, -56.0L / 9.0L, 11.0L / 16.0L};
        for (int m = 1; m <= 4; ++m) acc += a4[m - 1] * sinl(pi * k * m / (long double)g.n[a]);
      } else {
        for (int m = 1; m <= 3; ++m) acc += (long double)h->w.os[m] * sinl(pi * k * m / (long double)g.n[a]);
      }
      tv[3 * L + k - 1] = (double)acc;
    }
    double* d = nullptr;
    TRY(alloc_t(h, &d, 4LL * L));
    AHOC_HIP_TRY(hipMemcpyAsync(d, tv.data(), sizeof(double) * tv.size(), hipMemcpyHostToDevice, st));
    AHOC_HIP_TRY(hipStreamSynchronize(st));
    for (int r = 0; r < 4; ++r) tabs[4 * a + r] = d + (long long)r * L;
  }
  TRY(alloc_t(h, &h->pc, g.nq));
  TRY(alloc_t(h, &h->qc, g.nq));
  TRY(precond_symbol(g, h->wv, h->cshift, h->navier, tabs.data(), h->pc, h->qc, st, h->tri));
  if (h->p64.ready) {
    for (int a = 0; a < g.dim; ++a) h->ptb[a] = h->p64.tb[a];
    h->ptb_own = false;
  } else {
    h->ptb_own = true;
    for (int a = 0; a < g.dim; ++a) TRY(dst_tables_init<double>(h->ptb[a], g.n[a], st, &h->al));
  }
  AHOC_HIP_TRY(hipStreamSynchronize(st));
  return ST_OK;
}

// 2-D DST-I of every face block of a Q-layout vector, from x into y (y may equal x; the
// first pass of each face reads x, later ones work in place on y).  Faces x-, x+ hold
// [k][j], y-, y+ [k][i], z-, z+ [j][i] (lower axis fastest, no padding).  A square 2-D
// batch (N_x = N_y) is one row pass: its Q vector is 4 nb rows of N-1 entries.
int face_dst_q(ahoc_handle* h, const double* x, double* y, hipStream_t st) {
  const Geom& g = h->g;
  const DstTables<double>* tb = h->ptb;
  const long long ox = g.face_off[0], oy = g.face_off[2];
  if (g.dim == 3) {
    const long long oz = g.face_off[4];
    TRY(dst_pass<double>(tb[1], x + ox, y + ox, 2LL * g.ni[2], 1, g.ni[1], nullptr, 0, st));
    TRY(dst_pass<double>(tb[2], y + ox, y + ox, 2, g.ni[1], g.ni[1], nullptr, 0, st));
    TRY(dst_pass<double>(tb[0], x + oy, y + oy, 2LL * g.ni[2], 1, g.ni[0], nullptr, 0, st));
    TRY(dst_pass<double>(tb[2], y + oy, y + oy, 2, g.ni[0], g.ni[0], nullptr, 0, st));
    TRY(dst_pass<double>(tb[0], x + oz, y + oz, 2LL * g.ni[1], 1, g.ni[0], nullptr, 0, st));
    TRY(dst_pass<double>(tb[1], y + oz, y + oz, 2, g.ni[0], g.ni[0], nullptr, 0, st));
  } else if (g.n[0] == g.n[1] && g.nq == 4LL * g.ni[0]) {
    TRY(dst_pass<double>(tb[0], x, y, 4LL * g.nb, 1, g.ni[0], nullptr, 0, st));
  } else {  // each face line of every instance of a batch (instances nq apart)
    TRY(dst_pass<double>(tb[1], x + ox, y + ox, g.nb, 1, g.nq, nullptr, 0, st));
    TRY(dst_pass<double>(tb[1], x + ox + g.ni[1], y + ox + g.ni[1], g.nb, 1, g.nq, nullptr, 0, st));
    TRY(dst_pass<double>(tb[0], x + oy, y + oy, g.nb, 1, g.nq, nullptr, 0, st));
    TRY(dst_pass<double>(tb[0], x + oy + g.ni[0], y + oy + g.ni[0], g.nb, 1, g.nq, nullptr, 0, st));
  }
  return ST_OK;
}

// y = P^-1 v (FP64), y may not alias v
int precond_apply(ahoc_handle* h, const double* v, double* y, hipStream_t st) {
  const Geom& g = h->g;
  hipEvent_t e = tbegin(h, st);
  TRY(face_dst_q(h, v, y, st));
  TRY(precond_modes<double>(g, h->pc, h->qc, y, st));
  TRY(face_dst_q(h, y, y, st));
  tend(h, AHOC_K_PRECOND, e, (double)TQ(g) * 16.0, st);
  return ST_OK;
}

template <typename T> const T* q_in(ahoc_handle* h, Prec<T>& P, const double* q, hipStream_t st, int* rc) {
  if constexpr (sizeof(T) == 8) {
    (void)h; (void)P; (void)st;
    *rc = ST_OK;
    return reinterpret_cast<const T*>(q);
  } else {
    *rc = convert<double, float>(TQ(h->g), q, P.qT, st);
    return P.qT;
  }
}

// Triharmonic extension: the three chained Dirichlet solves from the face values Q of W
// (sources sw, sv, su of the W-, V- and U-solves, or none for the homogeneous form):
// W into P.bufA, V = L^-1(M W + sv) into P.bufB, then U = L^-1(M V + su) into P.bufA.
// Without sources the W-solve takes the spectral lift when the grid has it.
template <typename T>
int tri_fields(ahoc_handle* h, Prec<T>& P, const T* Q, const T* sw, const T* sv, const T* su, hipStream_t st) {
  if (!sw && P.spectral) TRY(vsolve_spec<T>(h, P, Q, st));
  else TRY(vsolve<T>(h, P, Q, sw, st));
  TRY(usolve<T>(h, P, Q, sv, st));
  hipEvent_t e = tbegin(h, st);
  TRY(rhs_u<T>(h->g, h->w, P.bufB, P.zq, P.ia, su, P.bufA, st));
  tend(h, AHOC_K_RHS_U, e, (double)sizeof(T) * (2.0 * h->g.nint + h->g.nnodal), st);
  return poisson<T>(h, P, P.bufA, P.scU, st);
}

template <typename T> int tri_gather(ahoc_handle* h, Prec<T>& P, const T* Q, const T* srcq, double* R, hipStream_t st) {
  hipEvent_t eg = tbegin(h, st);
  TRY(gather_tri<T>(h->g, P.bufA, Q, P.af, srcq, R, st));
  tend(h, AHOC_K_GATHER, eg, (double)h->g.nq * (5 * sizeof(T) + sizeof(double)), st);
  return ST_OK;
}

// y = S_h q  (homogeneous Lemma-1 form)
template <typename T> int matvec(ahoc_handle* h, Prec<T>& P, const double* q, double* y, hipStream_t st) {
  int rc = 0;
  hipEvent_t e = tbegin(h, st);
  const T* qT = q_in<T>(h, P, q, st, &rc);
  TRY(rc);
  if (h->tri) {
    TRY(tri_fields<T>(h, P, qT, nullptr, nullptr, nullptr, st));
    TRY(tri_gather<T>(h, P, qT, nullptr, y, st));
    tend(h, AHOC_K_MATVEC, e, (double)sizeof(T) * (34.0 * h->g.nint + 2.0 * h->g.nnodal), st);
    return ST_OK;
  }
  if (P.mspec) {
    TRY(matvec_mspec<T>(h, P, qT, y, st));
    // algorithmic bytes: generated pass (write 1), 3-D: y inverse (2), x pass (read, write:
    // 2, and the nodal 1/alpha), 3-D: y forward (2), slowest-axis forward (2), face reduction
    // (read 1)
    const double nv = h->g.dim == 3 ? 10.0 : 6.0;
    tend(h, AHOC_K_MATVEC, e, (double)sizeof(T) * (nv * h->g.nint + h->g.nnodal) * h->g.nb, st);
    return ST_OK;
  }
  if (P.spectral) {
    TRY(vsolve_spec<T>(h, P, qT, st));
    TRY(usolve_spec<T>(h, P, qT, nullptr, st));
    hipEvent_t eg = tbegin(h, st);
    TRY(gather_faces<T>(h->g, P.Fx, P.Fy, P.Fz, qT, P.af, nullptr, y, st));
    tend(h, AHOC_K_GATHER, eg, (double)TQ(h->g) * (3 * sizeof(T) + sizeof(double)), st);
  } else {
    TRY(vsolve<T>(h, P, qT, nullptr, st));
    TRY(usolve<T>(h, P, qT, nullptr, st));
    hipEvent_t eg = tbegin(h, st);
    TRY(gather<T>(h->g, h->w, P.bufB, qT, P.af, nullptr, y, st));
    tend(h, AHOC_K_GATHER, eg, (double)h->g.nq * (3 * sizeof(T) + 2 * sizeof(T) + sizeof(double)), st);
  }
  // algorithmic bytes of one matvec.  Spectral form: generated pass (write), 2 (3-D) or 1
  // (2-D) inverse passes, rhs_u (read V, 1/alpha, write), 2 or 1 forward passes, the
  // forward/scale pass and the face reduction (read).  Otherwise: lift, 10 or 6 passes,
  // rhs_u, gather.
  const double s = sizeof(T);
  const Geom& g = h->g;
  const double np = g.dim == 3 ? 2.0 : 1.0;
  const double vol = P.spectral ? (1.0 + 2.0 * np + 2.0 + 2.0 * np + 2.0 + 1.0) * g.nint + g.nnodal
                                : (1.0 + 2.0 * (2.0 * np + 1.0) * 2.0 + 2.0) * g.nint + g.nnodal;
  tend(h, AHOC_K_MATVEC, e, s * vol * g.nb, st);
  return ST_OK;
}

// b = -R(0) for sources (src_v, src_u, src_q) in precision T
template <typename T>
int schur_rhs(ahoc_handle* h, Prec<T>& P, const T* sv, const T* su, const T* sq, double* b, hipStream_t st) {
  if (h->tri) {
    if constexpr (sizeof(T) == 8) {
      TRY(tri_fields<T>(h, P, P.zq, sv, su, h->src_t, st));
      TRY(tri_gather<T>(h, P, P.zq, sq, h->R, st));
      return axpby(TQ(h->g), -1.0, h->R, 0.0, b, st);
    } else {
      return ST_UNSUPPORTED;
    }
  }
  TRY(vsolve<T>(h, P, P.zq, sv, st));
  if (P.spectral) {
    TRY(usolve_spec<T>(h, P, P.zq, su, st));
    TRY(gather_faces<T>(h->g, P.Fx, P.Fy, P.Fz, P.zq, P.af, sq, h->R, st));
  } else {
    TRY(usolve<T>(h, P, P.zq, su, st));
    TRY(gather<T>(h->g, h->w, P.bufB, P.zq, P.af, sq, h->R, st));
  }
  return axpby(TQ(h->g), -1.0, h->R, 0.0, b, st);
}

// Axes and pass kinds whose plain passes run as the matrix-core product, bit 2 axis + kind,
// for the operator of the solve's precision.
int gemm_mask(const ahoc_handle* h) {
  int m = 0;
  for (int a = 0; a < h->g.dim; ++a)
    for (int k = 0; k < 2; ++k) {
      const bool on = h->opt.precision == AHOC_MIXED ? (h->p32.ready && h->p32.tb[a].method[k] == DST_M_GEMM)
                                                     : (h->p64.ready && h->p64.tb[a].method[k] == DST_M_GEMM);
      if (on) m |= 1 << (2 * a + k);
    }
  return m;
}

double read_scalar(ahoc_handle* h, const double* dptr, hipStream_t st, int* rc) {
  hipError_t e = hipMemcpyAsync(h->pinned, dptr, sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    set_last_error(hipGetErrorString(e), "read_scalar");
    *rc = ST_HIP;
    return 0.0;
  }
  *rc = ST_OK;
  return h->pinned[0];
}

// Copy `count` doubles from the device into h->pinned and wait.
int read_vec(ahoc_handle* h, const double* dptr, int count, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(h->pinned, dptr, sizeof(double) * count, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    set_last_error(hipGetErrorString(e), "read_vec");
    return ST_HIP;
  }
  return ST_OK;
}

// Upload `count` ints from h->pinned_i (stream-ordered; the host buffer is reused only
// after the next synchronising read).
int write_ints(ahoc_handle* h, int* dptr, int count, hipStream_t st) {
  AHOC_HIP_TRY(hipMemcpyAsync(dptr, h->pinned_i, sizeof(int) * count, hipMemcpyHostToDevice, st));
  return ST_OK;
}

// Blocks per segment of a dot sweep: at least 2048 entries per block (8 per thread), so a
// short segment (a small 2-D batch instance) does not launch hundreds of idle blocks.
int dot_blocks(const ahoc_handle* h, long long n) {
  const long long b = (n + 2047) / 2048;
  return (int)std::max<long long>(1, std::min<long long>(h->nb_dot, b));
}

// Per-instance dot products of two batch vectors: out[2 s] = <a_s, b_s>.
int dot_dev(ahoc_handle* h, const double* a, const double* b, hipStream_t st, double* out) {
  const long long n = h->g.nq;
  const int nbk = dot_blocks(h, n);
  return mdot(a, n, 1, b, n, h->g.nb, h->part, nbk, out, 2, st);
}

double absmax(ahoc_handle* h, const void* x, bool dbl, long long n, hipStream_t st, int* rc) {
  const int nb = 1024;
  *rc = dbl ? absmax_partial<double>(n, (const double*)x, h->red, nb, st)
            : absmax_partial<float>(n, (const float*)x, h->red, nb, st);
  if (*rc) return 0.0;
  std::vector<double> hb(nb);
  hipError_t e = hipMemcpyAsync(hb.data(), h->red, sizeof(double) * nb, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    set_last_error(hipGetErrorString(e), "absmax");
    *rc = ST_HIP;
    return 0.0;
  }
  double m = 0;
  for (double v : hb) m = v > m ? v : m;
  return m;
}

struct GmresResult {
  int iters = 0;
  double relres = 0;
  bool converged = false;
};

// Restarted GMRES(m) on S_h x = b for every instance of the handle (lock-step over a
// batch: one matvec, one Arnoldi step and one host read of the residual estimates per
// iteration for all instances), from x = 0 or (x0) from the x passed in -- then the first
// cycle starts from the true residual b - S x --, right-preconditioned by the boundary
// symbol when it is enabled (x = P^-1 y, GMRES on S P^-1 y = b; the residual it monitors
// is the true one).  All vectors FP64 on the device.  An instance stops when its estimate
// reaches tol (its later basis vectors are zero and its Krylov dimension is frozen); with
// an FP32 operator it also stops once eight iterations gained less than a factor 2 (the
// estimate levels off at the operator's rounding level).  A non-finite ||b|| or residual
// estimate (NaN or Inf in the data) ends the instance as not converged.
// w = S_h P^-1 v (or S_h v without the preconditioner).  With use_graph the launches run
// as one captured HIP graph from the fixed buffers gin -> gout (the copies in and out are
// stream-ordered device copies outside the graph); the graph is captured on the second
// application (the first runs eagerly, so one-time kernel attribute queries happen outside
// the capture) and capture failures (e.g. on the legacy default stream) fall back to
// eager launches for the rest of the handle's life.
template <typename T>
int apply_op(ahoc_handle* h, Prec<T>& P, bool pre, const double* v, double* w, hipStream_t st) {
  const int pi = sizeof(T) == 8 ? 1 : 0;
  auto body = [&](const double* in, double* out) -> int {
    if (pre) {
      TRY(precond_apply(h, in, h->zvec, st));
      return matvec<T>(h, P, h->zvec, out, st);
    }
    return matvec<T>(h, P, in, out, st);
  };
  const bool graph = h->opt.use_graph && h->gin && !h->prof && !h->opg_failed[pi];
  if (graph && !h->opg[pi] && h->opg_uses[pi]++ >= 1) {
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    int rc = ST_OK;
    if (e == hipSuccess) {
      rc = body(h->gin, h->gout);
      const hipError_t e2 = hipStreamEndCapture(st, &gr);
      e = e2;
    }
    if (e == hipSuccess && rc == ST_OK && gr) e = hipGraphInstantiate(&h->opg[pi], gr, nullptr, nullptr, 0);
    if (gr) (void)hipGraphDestroy(gr);
    if (e != hipSuccess || rc != ST_OK || !h->opg[pi]) {
      (void)hipGetLastError();
      if (h->opg[pi]) (void)hipGraphExecDestroy(h->opg[pi]);
      h->opg[pi] = nullptr;
      h->opg_failed[pi] = true;
    }
  }
  if (graph && h->opg[pi]) {
    const long long n = TQ(h->g);
    AHOC_HIP_TRY(hipMemcpyAsync(h->gin, v, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    AHOC_HIP_TRY(hipGraphLaunch(h->opg[pi], st));
    ++h->graph_steps;
    AHOC_HIP_TRY(hipMemcpyAsync(w, h->gout, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    return ST_OK;
  }
  return body(v, w);
}

// AHOC_GMRES_CHECK=1: read the device state after every Arnoldi step (for comparisons).
bool check_every_step() {
  static const bool v = [] {
    const char* e = std::getenv("AHOC_GMRES_CHECK");
    return e && std::atoi(e) == 1;
  }();
  return v;
}

template <typename T>
int gmres(ahoc_handle* h, Prec<T>& P, const double* b, double* x, double tol, int max_iters,
          std::vector<GmresResult>& res, int* matvecs, hipStream_t st, bool x0 = false) {
  const bool inexact = sizeof(T) == 4;
  const bool pre = h->pc != nullptr;
  const int ns = h->g.nb;
  const long long nq = h->g.nq;
  const int nbk = dot_blocks(h, nq);
  const long long nt = nq * ns;  // batch vector length
  const int m = h->m;
  // device state per instance: [act | kk | nit | flag | hcnt] (see step_update)
  int* act = h->ist;
  int* kk = h->ist + ns;
  const int* hst = h->pinned_s;  // host image of [act | kk | nit | flag]
  res.assign(ns, GmresResult());
  std::vector<double> bnorm(ns);
  std::vector<char> conv(ns, 0);  // 0 iterating, 1 converged, 2 stopped without convergence
  if (!x0) TRY(fill(nt, 0.0, x, st));
  TRY(dot_dev(h, b, b, st, h->nrm));
  TRY(read_vec(h, h->nrm, 2 * ns, st));
  bool any = false;
  for (int s = 0; s < ns; ++s) {
    const double b2 = h->pinned[2 * s];
    bnorm[s] = std::sqrt(std::max(b2, 0.0));
    if (!std::isfinite(b2)) {  // NaN or Inf in the data: stop, not converged
      conv[s] = 2;
      res[s].converged = false;
      res[s].relres = b2;
      continue;
    }
    conv[s] = bnorm[s] > 0 ? 0 : 1;
    res[s].converged = conv[s] == 1;
    any = any || !conv[s];
  }
  if (!any) return ST_OK;
  for (int s = 0; s < ns; ++s) h->pinned_b[s] = bnorm[s] > 0 && std::isfinite(bnorm[s]) ? bnorm[s] : 1.0;
  AHOC_HIP_TRY(hipMemcpyAsync(h->bn, h->pinned_b, sizeof(double) * ns, hipMemcpyHostToDevice, st));
  TRY(fill_int(h->ist + 2 * ns, 3LL * ns, 0, st));  // nit, flag, hcnt
  std::vector<double> est_prev(ns, 0.0);
  bool first = !x0;
  while (true) {
    const double* r = b;
    if (!first) {
      TRY(matvec<T>(h, P, x, h->rvec, st));
      ++*matvecs;
      TRY(axpby(nt, 1.0, b, -1.0, h->rvec, st));  // r = b - S x
      r = h->rvec;
    }
    first = false;
    TRY(dot_dev(h, r, r, st, h->nrm));
    TRY(start_cycle(h->Vb, r, nq, ns, h->nrm, h->gv, m, h->beta, st));
    TRY(read_vec(h, h->beta, ns, st));
    any = false;
    for (int s = 0; s < ns; ++s) {
      h->pinned_i[s] = 0;
      h->pinned_i[ns + s] = 0;  // Krylov dimension of the cycle
      if (conv[s]) continue;
      res[s].relres = h->pinned[s] / bnorm[s];
      if (!std::isfinite(h->pinned[s])) {
        conv[s] = 2;
        continue;
      }
      if (h->pinned[s] <= tol * bnorm[s]) {
        conv[s] = 1;
        res[s].converged = true;
        continue;
      }
      if (res[s].iters >= max_iters) {
        conv[s] = 2;
        continue;
      }
      h->pinned_i[s] = 1;
      any = true;
    }
    if (!any) return ST_OK;
    TRY(write_ints(h, h->ist, 2 * ns, st));  // act, kk (the host buffer is reused after the next read)
    // The steps run without host reads; the host checks the device state after the step at
    // which the slowest active instance is predicted to converge (from its observed
    // contraction), at most 8 steps (and never past an iteration cap) apart.
    int jmax = 0, next = 0, jprev = -1;
    for (int j = 0; j < m; ++j) {
      double* vj = h->Vb + (long long)j * nt;
      double* w = h->Vb + (long long)(j + 1) * nt;
      TRY(apply_op<T>(h, P, pre, vj, w, st));
      ++*matvecs;
      hipEvent_t ek = tbegin(h, st);
      TRY(mdot(h->Vb, nt, j + 1, w, nq, ns, h->part, nbk, h->h1, m + 1, st));
      TRY(maxpy(w, h->Vb, nt, j + 1, h->h1, m + 1, -1.0, nq, ns, st));
      TRY(mdot(h->Vb, nt, j + 1, w, nq, ns, h->part, nbk, h->h2, m + 1, st));
      TRY(maxpy(w, h->Vb, nt, j + 1, h->h2, m + 1, -1.0, nq, ns, st));
      TRY(dot_dev(h, w, w, st, h->nrm));
      TRY(givens_update(ns, h->H, m, h->h1, h->h2, h->nrm, h->cs, h->sn, h->gv, j, h->resid, h->bn, tol, max_iters,
                        inexact, h->ist, h->hist, h->eres, st));
      TRY(scale_by_inv(w, nq, ns, h->resid, act, st));
      // CGS2: 2 x (j+1) dot sweeps and 2 x (j+1) axpy sweeps over the basis, plus norm and scale
      tend(h, AHOC_K_KRYLOV, ek, 8.0 * nt * (4.0 * (j + 1) + 2.0 * 2 + 3.0), st);
      jmax = j + 1;
      if (j < next && j < m - 1) continue;
      // one host round trip: [act | kk | nit | flag] and the last active estimates
      AHOC_HIP_TRY(hipMemcpyAsync(h->pinned_s, h->ist, sizeof(int) * 4 * ns, hipMemcpyDeviceToHost, st));
      TRY(read_vec(h, h->eres, ns, st));
      any = false;
      double need = 1.0;
      int cap = 8;
      for (int s = 0; s < ns; ++s) {
        if (conv[s]) continue;
        res[s].iters = hst[2 * ns + s];
        const double est = h->pinned[s];
        res[s].relres = est;
        if (hst[s]) {
          any = true;
          cap = std::min(cap, std::max(1, max_iters - res[s].iters));
          if (jprev >= 0 && est_prev[s] > est && est > 0) {
            const double rate = std::pow(est / est_prev[s], 1.0 / (j - jprev));
            need = std::max(need, std::log(tol / est) / std::log(rate));
          }
          est_prev[s] = est;
        } else if (hst[3 * ns + s] == 1) {
          conv[s] = 1;
          res[s].converged = true;
        }
      }
      if (!any) break;
      next = j + (check_every_step() ? 1 : std::max(1, std::min(cap, (int)std::floor(0.9 * need))));
      jprev = j;
    }
    TRY(back_solve(ns, h->H, m, h->gv, kk, jmax, h->y, st));
    if (pre) {  // x += P^-1 (V y); the cycle's residual vector is free again
      TRY(fill(nt, 0.0, h->rvec, st));
      TRY(maxpy(h->rvec, h->Vb, nt, jmax, h->y, m + 1, 1.0, nq, ns, st));
      TRY(precond_apply(h, h->rvec, h->zvec, st));
      TRY(axpby(nt, 1.0, h->zvec, 1.0, x, st));
    } else {
      TRY(maxpy(x, h->Vb, nt, jmax, h->y, m + 1, 1.0, nq, ns, st));
    }
    // another cycle for the instances that neither converged, stalled (flag 2) nor hit the
    // cap; the state is the last check's, taken after the cycle's last step
    any = false;
    for (int s = 0; s < ns; ++s) {
      if (conv[s]) continue;
      if (hst[3 * ns + s] == 2 || res[s].iters >= max_iters) conv[s] = 2;
      else any = true;
    }
    if (!any) return ST_OK;
  }
}

// Concatenate one nodal input field of `count` instances into a batch array (nullptr if no
// instance has it; instances without it get zeros).
int gather_field(ahoc_handle* h, const ahoc_problem* pbs, int count, size_t off, int slot, double** out,
                 hipStream_t st) {
  bool any = false;
  for (int i = 0; i < count; ++i)
    any = any || *reinterpret_cast<const double* const*>(reinterpret_cast<const char*>(&pbs[i]) + off);
  *out = nullptr;
  if (!any) return ST_OK;
  const long long nn = h->g.nnodal;
  TRY(alloc_t(h, out, nn * count));
  void** hp = h->ptab_host.data() + (size_t)slot * count;
  for (int i = 0; i < count; ++i)
    hp[i] = const_cast<double*>(
        *reinterpret_cast<const double* const*>(reinterpret_cast<const char*>(&pbs[i]) + off));
  AHOC_HIP_TRY(hipMemcpyAsync(h->ptab + (size_t)slot * count, hp, sizeof(void*) * count,
                              hipMemcpyHostToDevice, st));
  return gather_ptrs(reinterpret_cast<const double* const*>(h->ptab + (size_t)slot * count), nn, count, *out, st);
}

// Set up one problem, or a batch of `count` 2-D problems on the same grid (same n, lo, hi),
// whose arrays then hold the instances one after another.
int setup_impl(const ahoc_problem* pbs, int count, hipStream_t st, ahoc_handle* h) {
  Geom& g = h->g;
  const ahoc_problem* pb = &pbs[0];
  make_geom(pb, g);
  g.nb = count;
  make_weights(g, h->w);
  h->wv = h->w;
  h->m = h->opt.restart;
  h->tri = pb->equation == AHOC_TRIHARMONIC;
  if (h->tri) {
    if (count != 1) {
      set_last_error("triharmonic problems are set up one per handle", "ahoc_setup");
      return ST_UNSUPPORTED;
    }
    if (h->opt.precision == AHOC_MIXED && h->opt.refine != 1) {
      set_last_error("the triharmonic equation in MIXED precision needs refine = 1", "ahoc_setup");
      return ST_UNSUPPORTED;
    }
  }
  const double *alpha = pb->alpha, *f = pb->f, *gD = pb->gD, *gN = pb->gN, *lapgD = pb->lapgD, *gL = pb->gL;
  for (int i = 0; i < count; ++i)
    if (pbs[i].navier != pb->navier) {
      set_last_error("the instances of a batch must share their Navier faces", "ahoc_setup");
      return ST_UNSUPPORTED;
    }
  h->navier = pb->navier;
  if (count > 1) {
    double *a_, *f_, *gd_, *gn_, *lg_, *gl_ = nullptr;
    h->ptab_host.assign((size_t)7 * count, nullptr);
    TRY(alloc_t(h, &h->ptab, 7LL * count));
    TRY(gather_field(h, pbs, count, offsetof(ahoc_problem, alpha), 0, &a_, st));
    TRY(gather_field(h, pbs, count, offsetof(ahoc_problem, f), 1, &f_, st));
    TRY(gather_field(h, pbs, count, offsetof(ahoc_problem, gD), 2, &gd_, st));
    TRY(gather_field(h, pbs, count, offsetof(ahoc_problem, gN), 3, &gn_, st));
    TRY(gather_field(h, pbs, count, offsetof(ahoc_problem, lapgD), 4, &lg_, st));
    if (pb->navier) TRY(gather_field(h, pbs, count, offsetof(ahoc_problem, gL), 6, &gl_, st));
    alpha = a_, f = f_, gD = gd_, gN = gn_, lapgD = lg_, gL = gl_;
  }
  // FP64 data
  TRY(alloc_t(h, &h->ia64, TN(g)));
  TRY(alloc_t(h, &h->af64, TQ(g)));
  TRY(alloc_int(h, &h->src_v, st));
  TRY(alloc_t(h, &h->src_q, TQ(g)));
  if (gD) {
    TRY(alloc_int(h, &h->src_u, st));
    TRY(alloc_t(h, &h->gD, TN(g)));
    AHOC_HIP_TRY(hipMemcpyAsync(h->gD, gD, sizeof(double) * TN(g), hipMemcpyDeviceToDevice, st));
  }
  TRY(alloc_t(h, &h->red, 1024));
  TRY(alloc_t(h, &h->R, TQ(g)));
  const bool mixed = h->opt.precision == AHOC_MIXED;
  float* ia32 = nullptr;
  float* af32 = nullptr;
  if (mixed) {
    TRY(alloc_t(h, &ia32, TN(g)));
    TRY(alloc_t(h, &af32, TQ(g)));
  }
  if (h->tri) {
    // Delta^3 u = f: no coefficient (1/alpha = 1 in the weighting-operator kernels); the
    // sources of the W-, V- and U-solves and the q-rows' known part
    TRY(fill(TN(g), 1.0, h->ia64, st));
    if (ia32) TRY(convert<double, float>(TN(g), h->ia64, ia32, st));
    if (!h->src_u) TRY(alloc_int(h, &h->src_u, st));
    TRY(alloc_int(h, &h->src_t, st));
    TRY(tri_sources(g, h->w, f, gD, pb->lapu, pb->bilap, h->src_v, h->src_u, h->src_t, st));
    TRY(tri_srcq(g, h->navier, gD, gN, pb->gNN, pb->tang4, pb->bilap, h->src_q, h->af64, af32, st));
  } else {
    TRY(setup_inv_alpha(TN(g), alpha, h->ia64, ia32, h->red, 1024, st));
    {
      std::vector<double> hb(1024);
      AHOC_HIP_TRY(hipMemcpyAsync(hb.data(), h->red, sizeof(double) * 1024, hipMemcpyDeviceToHost, st));
      AHOC_HIP_TRY(hipStreamSynchronize(st));
      double mn = 1e300;
      for (double v : hb) mn = v < mn ? v : mn;
      if (!(mn > 0.0)) {
        set_last_error("alpha must be positive everywhere", "ahoc_setup");
        return ST_INVALID;
      }
      if (pb->beta_nodal) {
        if (count != 1 || h->opt.precision != AHOC_FP64) {
          set_last_error("a variable beta needs FP64 precision and a single problem per handle", "ahoc_setup");
          return ST_UNSUPPORTED;
        }
        h->cvar = true;
        h->opt.use_graph = 0;  // the BiCGSTAB V-solve reads its dot products on the host
        TRY(alloc_t(h, &h->cnod, TN(g)));
        TRY(mul(TN(g), pb->beta_nodal, h->ia64, h->cnod, st));
        TRY(minmax_partial(TN(g), h->cnod, h->red, 512, st));
        std::vector<double> hb(1024);
        AHOC_HIP_TRY(hipMemcpyAsync(hb.data(), h->red, sizeof(double) * 1024, hipMemcpyDeviceToHost, st));
        AHOC_HIP_TRY(hipStreamSynchronize(st));
        double cmin = 1e300, cmax = -1e300;
        for (int b = 0; b < 512; ++b) {
          cmin = std::min(cmin, hb[2 * b]);
          cmax = std::max(cmax, hb[2 * b + 1]);
        }
        h->cshift = 0.5 * (cmin + cmax);
        for (int a = 0; a < 3; ++a) h->wv.cf[a] = h->w.cf[a] - h->cshift * h->w.m1;
        {  // one block of seven interior vectors, TA(g) apart (the dot sweeps rely on it)
          double* blk = nullptr;
          TRY(alloc_t(h, &blk, 7 * TA(g)));
          AHOC_HIP_TRY(hipMemsetAsync(blk, 0, sizeof(double) * 7 * (size_t)TA(g), st));  // zero padding
          for (int k = 0; k < 7; ++k) h->bk[k] = blk + k * TA(g);
        }
        TRY(alloc_t(h, &h->bdot, 8));
        TRY(alloc_t(h, &h->bpart, 2LL * VS_DOT_BLOCKS));
        AHOC_HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&h->bpin), sizeof(double) * 8, hipHostMallocDefault));
      } else if (pb->beta != 0.0) {
        // the v-equation -L_h V + (beta/alpha) M V = M f is solved by the sine transforms only
        // for a constant shift beta/alpha
        int rc = 0;
        const double mx = absmax(h, alpha, true, TN(g), st, &rc);
        TRY(rc);
        if (count != 1 || mx - mn > 1e-14 * mx) {
          set_last_error("beta != 0 needs a constant alpha (and a single problem per handle)", "ahoc_setup");
          return ST_UNSUPPORTED;
        }
        if (h->opt.precision == AHOC_MIXED && h->opt.refine != 1) {
          set_last_error("beta != 0 in MIXED precision needs refine = 1", "ahoc_setup");
          return ST_UNSUPPORTED;
        }
        h->cshift = pb->beta / mx;
        for (int a = 0; a < 3; ++a) h->wv.cf[a] = h->w.cf[a] - h->cshift * h->w.m1;
      }
    }
    TRY(setup_face_alpha(g, alpha, h->af64, af32, st));
    TRY(setup_sources(g, h->w, f, alpha, gD, gN, lapgD, h->src_v, h->src_u, h->src_q, st));
    if (h->navier) TRY(setup_navier(g, h->navier, alpha, gL, h->af64, af32, h->src_q, st));
    if (lapgD) {
      // V = alpha * Delta u on edges and corners (Remark 1); read there only
      TRY(alloc_t(h, &h->vedge, TN(g)));
      TRY(mul(TN(g), alpha, lapgD, h->vedge, st));
    }
  }
  // FP64 machinery (plain solve, or the refinement's reference operators)
  h->p64.ia = h->ia64;
  h->p64.af = h->af64;
  const bool schur_ir = mixed && h->opt.refine == 1;
  if (!mixed || schur_ir) TRY(prec_init<double>(h, h->p64, h->opt.tile_fp64, st));
  if (h->cvar) {  // the V-solve is iterative: physical lift, U and gather
    h->p64.spectral = false;
    h->p64.mspec = false;
  }
  // the recovery's V-solve as the right-hand side's V (Q = 0) plus the homogeneous spectral
  // V-solve from Q: one FP64 array more
  if ((!mixed || schur_ir) && !h->tri && !h->cvar && h->p64.spectral) TRY(alloc_int(h, &h->V0, st));
  if (mixed) {
    h->p32.ia = ia32;
    h->p32.af = af32;
    TRY(prec_init<float>(h, h->p32, h->opt.tile_fp32, st));
    TRY(alloc_t(h, &h->Q64, TQ(g)));
    if (schur_ir) {
      TRY(alloc_t(h, &h->b64, TQ(g)));
    } else {
      TRY(alloc_int(h, &h->U64, st));
      TRY(alloc_int(h, &h->V64, st));
      TRY(alloc_int(h, &h->ru, st));
      TRY(alloc_int(h, &h->rv, st));
      TRY(alloc_t(h, &h->rq, TQ(g)));
    }
  }
  // Krylov workspace (per instance: Hessenberg, rotations, norms; one basis of batch vectors)
  const int m = h->m;
  const long long nb = g.nb;
  TRY(alloc_t(h, &h->Vb, (long long)(m + 1) * TQ(g)));
  TRY(alloc_t(h, &h->H, nb * (m + 1) * m));
  TRY(alloc_t(h, &h->cs, nb * m));
  TRY(alloc_t(h, &h->sn, nb * m));
  TRY(alloc_t(h, &h->gv, nb * (m + 1)));
  TRY(alloc_t(h, &h->h1, nb * (m + 1)));
  TRY(alloc_t(h, &h->h2, nb * (m + 1)));
  TRY(alloc_t(h, &h->nrm, 2 * nb));
  TRY(alloc_t(h, &h->resid, 2 * nb));
  TRY(alloc_t(h, &h->beta, nb));
  TRY(alloc_t(h, &h->y, nb * (m + 1)));
  TRY(alloc_t(h, &h->part, nb * (m + 1) * dot_blocks(h, g.nq)));
  TRY(alloc_t(h, &h->act, nb));
  TRY(alloc_t(h, &h->ist, 5 * nb));
  TRY(alloc_t(h, &h->hist, 16 * nb));
  TRY(alloc_t(h, &h->eres, nb));
  TRY(alloc_t(h, &h->bn, nb));
  TRY(alloc_t(h, &h->bvec, TQ(g)));
  TRY(alloc_t(h, &h->dq, TQ(g)));
  TRY(alloc_t(h, &h->rvec, TQ(g)));
  TRY(alloc_t(h, &h->zvec, TQ(g)));
  if (h->opt.use_graph) {
    TRY(alloc_t(h, &h->gin, TQ(g)));
    TRY(alloc_t(h, &h->gout, TQ(g)));
  }
  if (nb > 1) TRY(alloc_t(h, &h->ubuf, TN(g)));
  AHOC_HIP_TRY(hipMemsetAsync(h->H, 0, sizeof(double) * nb * (m + 1) * m, st));
  const size_t npin = (size_t)std::max<long long>(8, 2 * nb);
  AHOC_HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&h->pinned), sizeof(double) * npin, hipHostMallocDefault));
  AHOC_HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&h->pinned_i), sizeof(int) * npin, hipHostMallocDefault));
  AHOC_HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&h->pinned_s), sizeof(int) * 4 * nb, hipHostMallocDefault));
  AHOC_HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&h->pinned_b), sizeof(double) * nb, hipHostMallocDefault));
  AHOC_HIP_TRY(hipStreamSynchronize(st));
  if (h->opt.precond) TRY(precond_init(h, st));
  return ST_OK;
}

}  // namespace
}  // namespace ahoc

// ======================================================================================
// C ABI
// ======================================================================================

extern "C" {

void ahoc_default_options(ahoc_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = AHOC_FP64;
  o->restart = 30;
  o->max_iters = 2000;
  o->tol = 1e-12;
  o->inner_tol = 1e-5;
  o->sweep_tol = 1e-11;
  o->max_sweeps = 8;
  o->tile_fp64 = 0;
  o->tile_fp32 = 0;
  o->precond = 1;
  o->refine = 1;
  o->use_graph = 0;
}

const char* ahoc_status_string(ahoc_status s) {
  switch (s) {
    case AHOC_OK: return "ok";
    case AHOC_E_INVALID: return "invalid argument";
    case AHOC_E_NOMEM: return "out of device memory";
    case AHOC_E_NOCONV: return "not converged";
    case AHOC_E_HIP: return "HIP runtime error";
    case AHOC_E_UNSUPPORTED: return "unsupported size";
  }
  return "unknown status";
}

const char* ahoc_last_error(void) { return ahoc::g_err.c_str(); }

void ahoc_destroy(ahoc_handle* h) {
  if (!h) return;
  // the handle's last enqueued work (solves and setup return after completion; the
  // asynchronous entry points record done_ev on their stream), and pending timing events
  if (h->done_ev && h->done_rec) (void)hipEventSynchronize(h->done_ev);
  for (auto& p : h->pending) (void)hipEventSynchronize(p.b);
  ahoc::prec_free(h->p64);
  ahoc::prec_free(h->p32);
  if (h->ptb_own)
    for (int a = 0; a < 3; ++a) ahoc::dst_tables_free(h->ptb[a]);
  for (int i = 0; i < 2; ++i)
    if (h->opg[i]) (void)hipGraphExecDestroy(h->opg[i]);
  for (void* p : h->allocs) ahoc::dev_free(h->al, p);
  for (hipEvent_t e : h->evpool) (void)hipEventDestroy(e);
  if (h->done_ev) (void)hipEventDestroy(h->done_ev);
  if (h->pinned) (void)hipHostFree(h->pinned);
  if (h->pinned_i) (void)hipHostFree(h->pinned_i);
  if (h->pinned_s) (void)hipHostFree(h->pinned_s);
  if (h->pinned_b) (void)hipHostFree(h->pinned_b);
  if (h->bpin) (void)hipHostFree(h->bpin);
  delete h;
}

size_t ahoc_nq(const ahoc_handle* h) { return h ? (size_t)h->g.nq : 0; }

ahoc_status ahoc_copy_bandwidth(int pattern, const float* in, float* out, int nx, int ny, int nz, void* stream) {
  const int rc = ahoc::copy_bandwidth(pattern, in, out, nx, ny, nz, (hipStream_t)stream);
  if (rc == ahoc::ST_INVALID) ahoc::set_last_error("bad pattern, pointer or size (nx % 32)", "ahoc_copy_bandwidth");
  return (ahoc_status)rc;
}

ahoc_status ahoc_dst_choice(const ahoc_handle* h, int precision, int axis, int kind, int* method, int* tile,
                            double* t_default_us, double* t_gemm_us, double* t_best_us) {
  if (!h || !method || (precision != AHOC_FP64 && precision != AHOC_MIXED) || axis < 0 || axis >= h->g.dim ||
      (kind != 0 && kind != 1)) {
    ahoc::set_last_error("bad handle, precision, axis or kind", "ahoc_dst_choice");
    return AHOC_E_INVALID;
  }
  const bool dbl = precision == AHOC_FP64;
  if (dbl ? !h->p64.ready : !h->p32.ready) {
    ahoc::set_last_error("the handle has no operator in this precision", "ahoc_dst_choice");
    return AHOC_E_UNSUPPORTED;
  }
  auto get = [&](const auto& tb) {
    *method = tb.method[kind];
    if (tile) *tile = tb.method[kind] == DST_M_TILE ? tb.tile[kind] : 0;
    if (t_default_us) *t_default_us = tb.t_default_us[kind];
    if (t_gemm_us) *t_gemm_us = tb.t_gemm_us[kind];
    if (t_best_us) *t_best_us = tb.t_best_us[kind];
  };
  if (dbl) get(h->p64.tb[axis]);
  else get(h->p32.tb[axis]);
  return AHOC_OK;
}

static ahoc_status validate_problem(const ahoc_problem* pb) {
  if (pb->dim != 2 && pb->dim != 3) {
    ahoc::set_last_error("dim must be 2 or 3", "ahoc_setup");
    return AHOC_E_INVALID;
  }
  if (pb->equation != AHOC_BIHARMONIC && pb->equation != AHOC_TRIHARMONIC) {
    ahoc::set_last_error("equation must be AHOC_BIHARMONIC or AHOC_TRIHARMONIC", "ahoc_setup");
    return AHOC_E_INVALID;
  }
  const bool tri = pb->equation == AHOC_TRIHARMONIC;
  if (!pb->f || (!tri && !pb->alpha)) {
    ahoc::set_last_error(tri ? "f is required" : "alpha and f are required", "ahoc_setup");
    return AHOC_E_INVALID;
  }
  if (tri && (pb->beta != 0.0 || pb->beta_nodal)) {
    ahoc::set_last_error("the triharmonic equation has no beta term", "ahoc_setup");
    return AHOC_E_INVALID;
  }
  if (pb->navier & ~((1 << (2 * pb->dim)) - 1)) {
    ahoc::set_last_error("navier has a bit beyond the 2*dim faces", "ahoc_setup");
    return AHOC_E_INVALID;
  }
  for (int a = 0; a < pb->dim; ++a) {
    // the one-sided normal formula (Sec. 2.2) reads U_1, U_2, U_3 next to each face (the
    // triharmonic q-row U_1..U_4)
    if (pb->n[a] < (tri ? 5 : 4) || pb->n[a] > ahoc::DST_MAX_N || !(pb->hi[a] > pb->lo[a])) {
      ahoc::set_last_error(tri ? "need 5 <= n[a] <= 8192 and hi > lo" : "need 4 <= n[a] <= 8192 and hi > lo",
                           "ahoc_setup");
      return AHOC_E_INVALID;
    }
  }
  return AHOC_OK;
}

// count == 1: one problem; count > 1: a batch of 2-D problems on the same grid.
static ahoc_status setup_n(const ahoc_problem* pbs, int count, const ahoc_options* opt,
                           const ahoc_allocator* alloc, void* stream, ahoc_handle** out) {
  *out = nullptr;
  for (int i = 0; i < count; ++i) {
    const ahoc_status v = validate_problem(&pbs[i]);
    if (v != AHOC_OK) return v;
  }
  if (alloc && (!alloc->alloc || !alloc->free)) {
    ahoc::set_last_error("an allocator needs both alloc and free", "ahoc_setup");
    return AHOC_E_INVALID;
  }
  ahoc_options o;
  if (opt) o = *opt;
  else ahoc_default_options(&o);
  if (o.precision != AHOC_FP64 && o.precision != AHOC_MIXED) {
    ahoc::set_last_error("precision must be AHOC_FP64 or AHOC_MIXED", "ahoc_setup");
    return AHOC_E_INVALID;
  }
  if (o.restart < 1 || o.restart > 200) o.restart = 30;
  if (count > 1) o.refine = 1;  // a batch refines on the Schur system
  ahoc_handle* h = new ahoc_handle();
  h->opt = o;
  if (alloc) {
    h->al.alloc = alloc->alloc;
    h->al.free = alloc->free;
    h->al.ctx = alloc->ctx;
  }
  if (hipEventCreateWithFlags(&h->done_ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    h->done_ev = nullptr;
    ahoc::set_last_error("hipEventCreateWithFlags failed", "ahoc_setup");
    delete h;
    return AHOC_E_HIP;
  }
  const int rc = ahoc::setup_impl(pbs, count, (hipStream_t)stream, h);
  if (rc) {
    ahoc_destroy(h);
    return (ahoc_status)rc;
  }
  *out = h;
  return AHOC_OK;
}

ahoc_status ahoc_setup(const ahoc_problem* pb, const ahoc_options* opt, const ahoc_allocator* alloc, void* stream,
                       ahoc_handle** out) {
  if (!pb || !out) return AHOC_E_INVALID;
  return setup_n(pb, 1, opt, alloc, stream, out);
}

ahoc_status ahoc_schur_apply(ahoc_handle* h, const double* q, double* y, void* stream) {
  if (!h || !q || !y) return AHOC_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  int rc = h->opt.precision == AHOC_MIXED ? ahoc::matvec<float>(h, h->p32, q, y, st)
                                          : ahoc::matvec<double>(h, h->p64, q, y, st);
  if (!rc) rc = ahoc::mark_done(h, st);
  return (ahoc_status)rc;
}

ahoc_status ahoc_precond_apply(ahoc_handle* h, const double* q, double* y, void* stream) {
  if (!h || !q || !y) return AHOC_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  if (!h->pc) {
    ahoc::set_last_error("the handle was set up with precond = 0", "ahoc_precond_apply");
    return AHOC_E_INVALID;
  }
  if (q == y) {
    ahoc::set_last_error("q and y must not alias", "ahoc_precond_apply");
    return AHOC_E_INVALID;
  }
  int rc = ahoc::precond_apply(h, q, y, st);
  if (!rc) rc = ahoc::mark_done(h, st);
  return (ahoc_status)rc;
}

ahoc_status ahoc_schur_rhs(ahoc_handle* h, double* b, void* stream) {
  if (!h || !b) return AHOC_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if (h->opt.precision == AHOC_MIXED && h->opt.refine == 0) {
    // the coupled refinement's first sweep: the data in FP32 through the FP32 operator
    using namespace ahoc;
    rc = convert<double, float>(h->g.nalloc, h->src_v, h->rv, st);
    if (!rc && h->src_u) rc = convert<double, float>(h->g.nalloc, h->src_u, h->ru, st);
    if (!rc) rc = convert<double, float>(h->g.nq, h->src_q, h->rq, st);
    if (!rc) rc = schur_rhs<float>(h, h->p32, h->rv, h->src_u ? h->ru : nullptr, h->rq, b, st);
  } else {
    // FP64 operator: the FP64 solve, and the Schur refinement's b
    rc = ahoc::schur_rhs<double>(h, h->p64, h->src_v, h->src_u, h->src_q, b, st);
  }
  if (!rc) rc = ahoc::mark_done(h, st);
  return (ahoc_status)rc;
}

ahoc_status ahoc_poisson(ahoc_handle* h, const double* gin, double* wout, void* stream) {
  if (!h || !gin || !wout) return AHOC_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  using namespace ahoc;
  int rc;
  // dense caller arrays (row length n_x - 1) <-> padded interior rows
  const Geom& g = h->g;
  const long long rows = (long long)g.ni[1] * g.ni[2];
  if (h->opt.precision == AHOC_MIXED) {
    rc = pitch_copy<double, float>(rows, g.ni[0], gin, g.ni[0], h->p32.bufA, g.px, st);
    if (!rc) rc = poisson<float>(h, h->p32, h->p32.bufA, h->p32.scP, st);
    if (!rc) rc = pitch_copy<float, double>(rows, g.ni[0], h->p32.bufA, g.px, wout, g.ni[0], st);
  } else {
    rc = pitch_copy<double, double>(rows, g.ni[0], gin, g.ni[0], h->p64.bufA, g.px, st);
    if (!rc) rc = poisson<double>(h, h->p64, h->p64.bufA, h->p64.scP, st);
    if (!rc) rc = pitch_copy<double, double>(rows, g.ni[0], h->p64.bufA, g.px, wout, g.ni[0], st);
  }
  if (!rc) rc = mark_done(h, st);
  return (ahoc_status)rc;
}

}  // extern "C"

namespace ahoc {
namespace {

// Write the nodal U of every instance to its output (through the batch buffer for nb > 1).
int write_u(ahoc_handle* h, const double* Ui, double* const* u, hipStream_t st) {
  const Geom& g = h->g;
  if (g.nb == 1) return out_u<double>(g, Ui, h->gD, u[0], st);
  TRY(out_u<double>(g, Ui, h->gD, h->ubuf, st));
  void** hp = h->ptab_host.data() + 5 * (size_t)g.nb;
  for (int i = 0; i < g.nb; ++i) hp[i] = u[i];
  AHOC_HIP_TRY(hipMemcpyAsync(h->ptab + 5 * (size_t)g.nb, hp, sizeof(void*) * g.nb, hipMemcpyHostToDevice, st));
  return scatter_ptrs(h->ubuf, g.nnodal, g.nb, reinterpret_cast<double* const*>(h->ptab + 5 * (size_t)g.nb), st);
}

// Zero the segments (instances) of a batch vector whose flag in h->pinned_i is 0.
int zero_done(ahoc_handle* h, double* x, hipStream_t st) {
  const Geom& g = h->g;
  TRY(write_ints(h, h->act, g.nb, st));
  return zero_masked(x, g.nq, g.nb, h->act, st);
}

// u: one output per instance; v, q only for a single instance (nb = 1).  s: nb stats.
// With options.warm_start (single instance) q holds the initial guess on entry.
// During a solve the right-hand side's V (the V-solve with Q = 0) is kept in h->V0: the work
// array holding it and h->V0 trade places after the right-hand side and back when the solve
// returns, so that the Krylov steps (and any graph captured from them) always see the same
// work array.  The recovery's V-solve is then h->V0 plus the homogeneous spectral V-solve from
// Q (generation, inverse y and x passes, h->V0 added by the last pass) instead of a Poisson
// solve with the source.
struct KeepV0 {
  double*& a;
  double*& b;
  const bool on;
  KeepV0(ahoc_handle* h, Prec<double>& P)
      : a(P.bufA), b(h->V0), on(h->V0 != nullptr && P.spectral && !h->tri && !h->cvar) {
    if (on) std::swap(a, b);
  }
  ~KeepV0() {
    if (on) std::swap(a, b);
  }
};
int vsolve_rec(ahoc_handle* h, Prec<double>& P, const double* Q, const KeepV0& k, hipStream_t st) {
  return k.on ? vsolve_spec<double>(h, P, Q, st, false, false, h->V0) : vsolve<double>(h, P, Q, h->src_v, st);
}

int solve_fp64(ahoc_handle* h, double* const* u, double* v, double* q, ahoc_stats* s, hipStream_t st) {
  Prec<double>& P = h->p64;
  const Geom& g = h->g;
  std::vector<GmresResult> gr;
  int mv = 0;
  const bool warm = h->opt.warm_start && q && g.nb == 1;
  if (warm) AHOC_HIP_TRY(hipMemcpyAsync(h->dq, q, sizeof(double) * g.nq, hipMemcpyDeviceToDevice, st));
  TRY(schur_rhs<double>(h, P, h->src_v, h->src_u, h->src_q, h->bvec, st));
  const KeepV0 keep(h, P);
  TRY(gmres<double>(h, P, h->bvec, h->dq, h->opt.tol, h->opt.max_iters, gr, &mv, st, warm));
  if (h->tri) {
    TRY(tri_fields<double>(h, P, h->dq, h->src_v, h->src_u, h->src_t, st));
    TRY(write_u(h, P.bufA, u, st));
  } else {
    TRY(vsolve_rec(h, P, h->dq, keep, st));
    TRY(usolve<double>(h, P, h->dq, h->src_u, st));
    TRY(write_u(h, P.bufB, u, st));
  }
  if (v) TRY(out_v<double>(g, P.bufA, h->dq, h->vedge, v, st));
  if (q) AHOC_HIP_TRY(hipMemcpyAsync(q, h->dq, sizeof(double) * g.nq, hipMemcpyDeviceToDevice, st));
  AHOC_HIP_TRY(hipStreamSynchronize(st));
  bool all = true;
  for (int i = 0; i < g.nb; ++i) {
    s[i].converged = gr[i].converged;
    s[i].gmres_iters = gr[i].iters;
    s[i].sweeps = 1;
    s[i].matvecs = mv;
    s[i].schur_relres = gr[i].relres;
    s[i].last_update = 0;
    all = all && gr[i].converged;
  }
  return all ? ST_OK : ST_NOCONV;
}

// Mixed precision, refinement on the Schur system: b and the residual r = b - S_h Q are
// FP64 (FP64 operator), each correction S_h dQ = r is solved by GMRES with the FP32
// operator (FP64 Krylov basis, Arnoldi, Givens), Q is updated in FP64, and the final
// recovery of V and U from Q runs in FP64.  An instance stops when ||r|| <= tol ||b||
// (its residual is then zeroed, so later sweeps leave it alone).  The sweep predicted to be
// the last takes its residual from the recovery itself (r = -R(Q)), so a converged solve
// runs no FP64 Schur matvec after its last correction.
int solve_mixed_schur(ahoc_handle* h, double* const* u, double* v, double* q, ahoc_stats* s, hipStream_t st) {
  Prec<float>& P = h->p32;
  Prec<double>& D = h->p64;
  const Geom& g = h->g;
  const int nb = g.nb;
  int rc = 0;
  TRY(schur_rhs<double>(h, D, h->src_v, h->src_u, h->src_q, h->b64, st));
  const KeepV0 keep(h, D);
  TRY(dot_dev(h, h->b64, h->b64, st, h->nrm));
  TRY(read_vec(h, h->nrm, 2 * nb, st));
  std::vector<double> bnorm(nb), relres(nb, 0.0);
  std::vector<int> sweeps(nb, 0), iters(nb, 0);
  // conv: 0 refining, 1 converged, 2 stopped without convergence (non-finite data)
  std::vector<char> conv(nb, 0);
  bool all = true;
  for (int i = 0; i < nb; ++i) {
    const double b2 = h->pinned[2 * i];
    bnorm[i] = std::sqrt(std::max(b2, 0.0));
    if (!std::isfinite(b2)) {
      conv[i] = 2;
      relres[i] = b2;
    } else {
      conv[i] = bnorm[i] > 0 ? 0 : 1;
      relres[i] = conv[i] ? 0.0 : 1.0;
    }
    all = all && conv[i];
  }
  int mv = 0;
  const bool warm = h->opt.warm_start && q && nb == 1;
  if (warm) {
    // start from the caller's Q_0: first residual b - S_h Q_0 with the FP64 operator
    AHOC_HIP_TRY(hipMemcpyAsync(h->Q64, q, sizeof(double) * g.nq, hipMemcpyDeviceToDevice, st));
    TRY(matvec<double>(h, D, h->Q64, h->bvec, st));
    ++mv;
    TRY(axpby(TQ(g), 1.0, h->b64, -1.0, h->bvec, st));
    if (!all) {
      TRY(dot_dev(h, h->bvec, h->bvec, st, h->nrm));
      TRY(read_vec(h, h->nrm, 2, st));
      const double r2 = h->pinned[0];
      relres[0] = std::sqrt(std::max(r2, 0.0)) / bnorm[0];
      if (!std::isfinite(r2)) conv[0] = 2;
      else if (relres[0] <= h->opt.tol) conv[0] = 1;
      all = conv[0] != 0;
    }
  } else {
    TRY(fill(TQ(g), 0.0, h->Q64, st));
    AHOC_HIP_TRY(hipMemcpyAsync(h->bvec, h->b64, sizeof(double) * TQ(g), hipMemcpyDeviceToDevice, st));
  }
  double upd = 0;
  bool recovered = false;     // D.bufA / D.bufB hold V, U of the current Q64
  bool recover_check = true;  // cleared once a recovery-based check has not converged
  for (int sw = 0; sw < h->opt.max_sweeps && !all; ++sw) {
    std::vector<GmresResult> gr;
    TRY(gmres<float>(h, P, h->bvec, h->dq, h->opt.inner_tol, h->opt.max_iters, gr, &mv, st));
    // this sweep is predicted to converge when its GMRES reduction times the current
    // relative residual reaches the tolerance for every active instance
    bool predict = recover_check;
    for (int i = 0; i < nb; ++i)
      if (!conv[i]) predict = predict && gr[i].relres * relres[i] <= h->opt.tol;
    for (int i = 0; i < nb; ++i)
      if (!conv[i]) {
        iters[i] += gr[i].iters;
        ++sweeps[i];
      }
    TRY(axpby(TQ(g), 1.0, h->dq, 1.0, h->Q64, st));
    const double dn = absmax(h, h->dq, true, TQ(g), st, &rc);
    TRY(rc);
    const double qn = absmax(h, h->Q64, true, TQ(g), st, &rc);
    TRY(rc);
    upd = qn > 0 ? dn / qn : 0.0;
    // FP64 residual of the Schur system at the updated Q.  By Lemma 1 with the data,
    // b - S_h Q = -R(Q), R the boundary residual of the solution recovered from Q: when the
    // sweep is predicted to converge, the FP64 recovery of V and U (which the output needs
    // anyway) and the gather give it, instead of an FP64 Schur matvec before the recovery.
    hipEvent_t er = tbegin(h, st);
    if (predict) {
      if (h->tri) {
        TRY(tri_fields<double>(h, D, h->Q64, h->src_v, h->src_u, h->src_t, st));
        TRY(tri_gather<double>(h, D, h->Q64, h->src_q, h->R, st));
      } else {
        TRY(vsolve_rec(h, D, h->Q64, keep, st));
        TRY(usolve<double>(h, D, h->Q64, h->src_u, st));
        TRY(gather<double>(g, h->w, D.bufB, h->Q64, D.af, h->src_q, h->R, st));
      }
      TRY(axpby(TQ(g), -1.0, h->R, 0.0, h->bvec, st));
      recovered = true;
    } else {
      TRY(matvec<double>(h, D, h->Q64, h->bvec, st));
      ++mv;
      TRY(axpby(TQ(g), 1.0, h->b64, -1.0, h->bvec, st));
      recovered = false;
    }
    TRY(dot_dev(h, h->bvec, h->bvec, st, h->nrm));
    TRY(read_vec(h, h->nrm, 2 * nb, st));
    tend(h, AHOC_K_RESID, er, 8.0 * (double)TQ(g) * 4.0, st);
    all = true;
    for (int i = 0; i < nb; ++i) {
      if (!conv[i]) {
        const double r2 = h->pinned[2 * i];
        relres[i] = std::sqrt(std::max(r2, 0.0)) / bnorm[i];
        if (!std::isfinite(r2)) conv[i] = 2;
        else conv[i] = relres[i] <= h->opt.tol ? 1 : 0;
      }
      h->pinned_i[i] = !conv[i];
      all = all && conv[i];
    }
    if (predict && !all) recover_check = false;
    if (!all && nb > 1) TRY(zero_done(h, h->bvec, st));
  }
  if (!recovered) {
    if (h->tri) {
      TRY(tri_fields<double>(h, D, h->Q64, h->src_v, h->src_u, h->src_t, st));
    } else {
      TRY(vsolve_rec(h, D, h->Q64, keep, st));
      TRY(usolve<double>(h, D, h->Q64, h->src_u, st));
    }
  }
  TRY(write_u(h, h->tri ? D.bufA : D.bufB, u, st));
  if (v) TRY(out_v<double>(g, D.bufA, h->Q64, h->vedge, v, st));
  if (q) AHOC_HIP_TRY(hipMemcpyAsync(q, h->Q64, sizeof(double) * g.nq, hipMemcpyDeviceToDevice, st));
  AHOC_HIP_TRY(hipStreamSynchronize(st));
  bool ok = true;
  for (int i = 0; i < nb; ++i) {
    s[i].converged = conv[i] == 1;
    s[i].gmres_iters = iters[i];
    s[i].sweeps = sweeps[i];
    s[i].matvecs = mv;
    s[i].schur_relres = relres[i];
    s[i].last_update = upd;
    ok = ok && conv[i] == 1;
  }
  return ok ? ST_OK : ST_NOCONV;
}

// Mixed precision, refinement on the coupled system: the FP64 residual of the whole
// augmented system (u-, v- and q-rows) drives each sweep; the correction (Schur solve
// and recovery) runs with the FP32 operators and is accumulated into FP64 U, V, Q.
int solve_mixed(ahoc_handle* h, double* const* uo, double* v, double* q, ahoc_stats* s, hipStream_t st) {
  if (h->opt.refine == 1) return solve_mixed_schur(h, uo, v, q, s, st);
  if (h->g.nb != 1) return ST_INVALID;
  if (h->opt.warm_start && q) {
    set_last_error("warm_start needs the Schur refinement (refine = 1) in MIXED precision", "ahoc_solve");
    return ST_UNSUPPORTED;
  }
  double* u = uo[0];
  Prec<float>& P = h->p32;
  const Geom& g = h->g;
  int rc = 0;
  TRY(fill(g.nalloc, 0.0, h->U64, st));
  TRY(fill(g.nalloc, 0.0, h->V64, st));
  TRY(fill(g.nq, 0.0, h->Q64, st));
  int iters = 0, mv = 0, sweeps = 0;
  double prev = 0, upd = 0, relres = 0;
  bool conv = false;
  for (int sw = 0; sw < h->opt.max_sweeps; ++sw) {
    // residual of the coupled system at the current FP64 state (the data itself at sweep 0)
    const float* su = h->ru;
    if (sw == 0) {
      TRY(convert<double, float>(g.nalloc, h->src_v, h->rv, st));
      if (h->src_u) TRY(convert<double, float>(g.nalloc, h->src_u, h->ru, st));
      else su = nullptr;
      TRY(convert<double, float>(g.nq, h->src_q, h->rq, st));
    } else {
      hipEvent_t er = tbegin(h, st);
      TRY(resid64<float>(g, h->w, h->U64, h->V64, h->Q64, h->ia64, h->af64, h->src_u, h->src_v,
                         h->src_q, h->ru, h->rv, h->rq, st));
      tend(h, AHOC_K_RESID, er, 8.0 * (3.0 * g.nint + g.nnodal) + 4.0 * 2.0 * g.nint, st);
    }
    // correction: Schur solve in FP32 operators with FP64 Krylov, then recovery
    std::vector<GmresResult> grv;
    TRY(schur_rhs<float>(h, P, h->rv, su, h->rq, h->bvec, st));
    TRY(gmres<float>(h, P, h->bvec, h->dq, h->opt.inner_tol, h->opt.max_iters, grv, &mv, st));
    const GmresResult& gr = grv[0];
    iters += gr.iters;
    relres = gr.relres;
    TRY(convert<double, float>(g.nq, h->dq, P.qT, st));
    TRY(vsolve<float>(h, P, P.qT, h->rv, st));
    TRY(usolve<float>(h, P, P.qT, su, st));
    TRY(accumulate<float>(g.nalloc, P.bufB, h->U64, st));
    TRY(accumulate<float>(g.nalloc, P.bufA, h->V64, st));
    TRY(accumulate<double>(g.nq, h->dq, h->Q64, st));
    ++sweeps;
    const double du = absmax(h, P.bufB, false, g.nalloc, st, &rc);
    TRY(rc);
    const double un = absmax(h, h->U64, true, g.nalloc, st, &rc);
    TRY(rc);
    upd = un > 0 ? du / un : 0.0;
    // Remaining change of U after this sweep, estimated as upd * rho / (1 - rho) with the
    // contraction rho no smaller than the inner solve's achieved relative residual (the
    // first sweep's update is the whole solution, so its ratio says nothing about rho).
    if (upd <= h->opt.sweep_tol * 1e-3) {
      conv = true;
      break;
    }
    if (sw > 0) {
      double rho = gr.relres;
      if (sw > 1 && prev > 0) rho = std::max(rho, upd / prev);
      if (rho < 1.0 && upd * rho / (1.0 - rho) <= h->opt.sweep_tol) {
        conv = true;
        break;
      }
    }
    prev = upd;
  }
  TRY(out_u<double>(g, h->U64, h->gD, u, st));
  if (v) TRY(out_v<double>(g, h->V64, h->Q64, h->vedge, v, st));
  if (q) AHOC_HIP_TRY(hipMemcpyAsync(q, h->Q64, sizeof(double) * g.nq, hipMemcpyDeviceToDevice, st));
  AHOC_HIP_TRY(hipStreamSynchronize(st));
  s->converged = conv;
  s->gmres_iters = iters;
  s->sweeps = sweeps;
  s->matvecs = mv;
  s->schur_relres = relres;
  s->last_update = upd;
  return conv ? ST_OK : ST_NOCONV;
}

}  // namespace
}  // namespace ahoc

extern "C" {

ahoc_status ahoc_solve(ahoc_handle* h, double* u, double* v, double* q, ahoc_stats* stats, void* stream) {
  if (!h || !u) return AHOC_E_INVALID;
  ahoc_stats local;
  std::memset(&local, 0, sizeof(local));
  hipStream_t st = (hipStream_t)stream;
  const auto t0 = std::chrono::steady_clock::now();
  if (h->g.nb != 1) return AHOC_E_INVALID;
  if (h->tri && v) {
    ahoc::set_last_error("the triharmonic solve returns u and q only (v must be NULL)", "ahoc_solve");
    return AHOC_E_UNSUPPORTED;
  }
  double* const uo[1] = {u};
  const long long g0 = h->graph_steps, v0 = h->vs_iters;
  h->vs_worst = 0;
  int rc = h->opt.precision == AHOC_MIXED ? ahoc::solve_mixed(h, uo, v, q, &local, st)
                                          : ahoc::solve_fp64(h, uo, v, q, &local, st);
  local.graph_steps = (int)(h->graph_steps - g0);
  local.vsolve_iters = (int)(h->vs_iters - v0);
  local.vsolve_relres = h->vs_worst;
  if (rc == AHOC_OK && h->vs_worst > ahoc::VSOLVE_RELRES_MAX) {
    ahoc::set_last_error("a BiCGSTAB V-solve stopped above the residual bound (operator inexact)", "ahoc_solve");
    local.converged = 0;
    rc = AHOC_E_NOCONV;
  }
  (void)ahoc::mark_done(h, st);
  local.dst_gemm = ahoc::gemm_mask(h);
  const auto t1 = std::chrono::steady_clock::now();
  local.t_solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  if (stats) *stats = local;
  if (h->prof) {
    (void)hipStreamSynchronize(st);
    ahoc::tresolve(h);
  }
  return (ahoc_status)rc;
}

ahoc_status ahoc_set_dst_variant(int variant) {
  if (variant < 0 || variant > 5) return AHOC_E_INVALID;
  ahoc::dst_set_variant(variant);
  return AHOC_OK;
}

ahoc_status ahoc_set_dst_tile(int pass, int precision, int pairs) {
  if (precision != AHOC_FP64 && precision != AHOC_MIXED) return AHOC_E_INVALID;
  const int rc = ahoc::dst_set_tile(pass, precision == AHOC_FP64 ? 8 : 4, pairs);
  return rc == ahoc::ST_OK ? AHOC_OK : AHOC_E_INVALID;
}

ahoc_status ahoc_profile(ahoc_handle* h, int enable) {
  if (!h) return AHOC_E_INVALID;
  ahoc::tresolve(h);
  for (int k = 0; k < AHOC_NKIND; ++k) {
    h->kms[k] = 0;
    h->kcnt[k] = 0;
    h->kbytes[k] = 0;
  }
  h->prof = enable != 0;
  return AHOC_OK;
}

ahoc_status ahoc_kernel_times(ahoc_handle* h, int kind, double* total_ms, long long* launches,
                              double* bytes_per_launch) {
  if (!h || kind < 0 || kind >= AHOC_NKIND) return AHOC_E_INVALID;
  ahoc::tresolve(h);
  if (total_ms) *total_ms = h->kms[kind];
  if (launches) *launches = h->kcnt[kind];
  if (bytes_per_launch) *bytes_per_launch = h->kcnt[kind] ? h->kbytes[kind] / (double)h->kcnt[kind] : 0.0;
  return AHOC_OK;
}

ahoc_status ahoc_solve_batched(int count, const ahoc_problem* probs, const ahoc_options* opt,
                               const ahoc_allocator* alloc, double* const* u, ahoc_stats* stats, void* stream) {
  if (count < 0 || (count > 0 && (!probs || !u))) return AHOC_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  // Jobs: buckets of 2-D problems on the same grid run as one batch (lock-step GMRES, one
  // launch per kernel for all instances, chunks of about 64 M grid nodes); 3-D problems and
  // grids that occur once run alone.
  std::map<std::vector<double>, std::vector<int>> buckets;
  std::vector<std::vector<int>> jobs;
  for (int i = 0; i < count; ++i) {
    const ahoc_problem& p = probs[i];
    if (p.dim != 2 || !u[i] || p.beta != 0.0 || p.beta_nodal || p.equation != AHOC_BIHARMONIC) {  // alone
      jobs.push_back({i});
      continue;
    }
    // equal grids and equal Navier faces share a batch (and its preconditioner)
    buckets[{(double)p.n[0], (double)p.n[1], p.lo[0], p.lo[1], p.hi[0], p.hi[1], (double)p.navier}].push_back(i);
  }
  const long long node_budget = 64LL << 20;
  for (auto& kv : buckets) {
    const std::vector<int>& idx = kv.second;
    const long long nodes = (long long)(probs[idx[0]].n[0] + 1) * (probs[idx[0]].n[1] + 1);
    const size_t chunk = (size_t)std::max<long long>(1, std::min<long long>(4096, node_budget / nodes));
    for (size_t c0 = 0; c0 < idx.size(); c0 += chunk)
      jobs.emplace_back(idx.begin() + c0, idx.begin() + std::min(idx.size(), c0 + chunk));
  }
  // largest jobs first, so that the small ones fill in behind them
  auto work = [&](const std::vector<int>& jb) {
    const ahoc_problem& p = probs[jb[0]];
    long long nodes = 1;
    for (int a = 0; a < p.dim; ++a) nodes *= (long long)p.n[a] + 1;
    return nodes * (long long)jb.size();
  };
  std::stable_sort(jobs.begin(), jobs.end(),
                   [&](const std::vector<int>& a, const std::vector<int>& b) { return work(a) > work(b); });
  const int njobs = (int)jobs.size();
  if (njobs == 0) return AHOC_OK;

  // Jobs run concurrently, one host thread and one non-blocking stream per worker, so that
  // the per-iteration host round trips and short launches of one job overlap the others.
  int nworkers = 4;
  if (const char* e = std::getenv("AHOC_BATCH_STREAMS")) nworkers = std::atoi(e);
  nworkers = std::max(1, std::min(nworkers, std::min(njobs, 16)));
  std::vector<hipStream_t> ws(nworkers, nullptr);
  hipEvent_t ready = nullptr;
  int dev = 0;
  {
    hipError_t e = hipGetDevice(&dev);  // the workers run on the caller's current device
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ready, st);  // inputs written on the caller's stream
    for (int w = 0; w < nworkers && e == hipSuccess; ++w) {
      e = hipStreamCreateWithFlags(&ws[w], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipStreamWaitEvent(ws[w], ready, 0);
    }
    if (e != hipSuccess) {
      ahoc::set_last_error(hipGetErrorString(e), "ahoc_solve_batched");
      for (hipStream_t s : ws)
        if (s) (void)hipStreamDestroy(s);
      if (ready) (void)hipEventDestroy(ready);
      return AHOC_E_HIP;
    }
  }
  // ahoc_destroy synchronises the device, which would stall the other workers (and is not
  // allowed while another worker captures its GMRES operator graph): handles are kept until
  // every worker has finished.  A batch whose handles would exceed the memory budget (about
  // 128 B per grid node) destroys each handle after its job instead, without graphs.
  const size_t keep_budget = (size_t)48 << 30;
  double est = 0;
  for (const std::vector<int>& jb : jobs) est += 128.0 * (double)work(jb);
  const bool keep_all = est <= (double)keep_budget;
  ahoc_options jopt;
  if (opt) jopt = *opt;
  else ahoc_default_options(&jopt);
  if (!keep_all) jopt.use_graph = 0;
  std::vector<ahoc_status> jrc(njobs, AHOC_OK);
  std::vector<std::string> jerr(njobs);
  std::vector<ahoc_handle*> kept;
  size_t kept_bytes = 0;
  std::mutex mu;
  std::atomic<int> next{0};
  auto worker = [&](int w) {
    const hipStream_t s = ws[w];
    const bool dev_ok = hipSetDevice(dev) == hipSuccess;
    for (int jn = next++; jn < njobs; jn = next++) {
      if (!dev_ok) {
        jrc[jn] = AHOC_E_HIP;
        jerr[jn] = "ahoc_solve_batched: hipSetDevice failed in a worker thread";
        continue;
      }
      const std::vector<int>& jb = jobs[jn];
      const int k = (int)jb.size();
      std::vector<ahoc_problem> sub(k);
      std::vector<double*> uo(k);
      std::vector<ahoc_stats> so(k);
      for (int j = 0; j < k; ++j) {
        sub[j] = probs[jb[j]];
        uo[j] = u[jb[j]];
        std::memset(&so[j], 0, sizeof(ahoc_stats));
      }
      const auto t0 = std::chrono::steady_clock::now();
      ahoc_handle* h = nullptr;
      ahoc_status rc = setup_n(sub.data(), k, &jopt, alloc, s, &h);
      if (rc == AHOC_OK) {
        rc = (ahoc_status)(h->opt.precision == AHOC_MIXED
                               ? ahoc::solve_mixed(h, uo.data(), nullptr, nullptr, so.data(), s)
                               : ahoc::solve_fp64(h, uo.data(), nullptr, nullptr, so.data(), s));
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess && rc == AHOC_OK) {
          ahoc::set_last_error(hipGetErrorString(e), "ahoc_solve_batched");
          rc = AHOC_E_HIP;
        }
        if (h->cvar) {
          for (int j = 0; j < k; ++j) so[j].vsolve_relres = h->vs_worst;
          if (rc == AHOC_OK && h->vs_worst > ahoc::VSOLVE_RELRES_MAX) {
            for (int j = 0; j < k; ++j) so[j].converged = 0;
            ahoc::set_last_error("a BiCGSTAB V-solve stopped above the residual bound", "ahoc_solve_batched");
            rc = AHOC_E_NOCONV;
          }
        }
      }
      const double ms =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      for (int j = 0; j < k; ++j) {
        so[j].t_solve_ms = ms;  // wall time of the whole job (setup included)
        so[j].graph_steps = h ? (int)h->graph_steps : 0;
        so[j].dst_gemm = h ? ahoc::gemm_mask(h) : 0;
        if (stats) stats[jb[j]] = so[j];
      }
      jrc[jn] = rc;
      if (rc != AHOC_OK) jerr[jn] = ahoc::g_err;
      if (h) {
        bool keep = false;
        {
          std::lock_guard<std::mutex> lk(mu);
          if (keep_all || kept_bytes + h->dev_bytes <= keep_budget) {
            kept.push_back(h);
            kept_bytes += h->dev_bytes;
            keep = true;
          }
        }
        if (!keep) ahoc_destroy(h);
      }
    }
  };
  if (nworkers == 1) {
    worker(0);
  } else {
    std::vector<std::thread> th;
    for (int w = 0; w < nworkers; ++w) th.emplace_back(worker, w);
    for (std::thread& t : th) t.join();
  }
  for (ahoc_handle* h : kept) ahoc_destroy(h);
  for (hipStream_t s : ws) (void)hipStreamDestroy(s);
  (void)hipEventDestroy(ready);
  // first failing job in the order of the instances
  int first = -1;
  for (int jn = 0; jn < njobs; ++jn)
    if (jrc[jn] != AHOC_OK && (first < 0 || jobs[jn][0] < jobs[first][0])) first = jn;
  if (first < 0) return AHOC_OK;
  ahoc::g_err = jerr[first];
  return jrc[first];
}

ahoc_status ahoc_dst1(int precision, int dim, const int* nint, int axis, const void* in, void* out,
                      void* stream) {
  using namespace ahoc;
  if (!nint || !in || !out || (dim != 2 && dim != 3) || axis < 0 || axis >= dim) return AHOC_E_INVALID;
  long long ni[3] = {1, 1, 1};
  for (int a = 0; a < dim; ++a) {
    if (nint[a] < 1) return AHOC_E_INVALID;
    ni[a] = nint[a];
  }
  const int N = (int)ni[axis] + 1;
  if (!dst_supported(N)) return AHOC_E_UNSUPPORTED;
  long long inner = 1, outer = 1;
  for (int a = 0; a < axis; ++a) inner *= ni[a];
  for (int a = axis + 1; a < 3; ++a) outer *= ni[a];
  if (axis == 0) {
    outer = ni[1] * ni[2];
    inner = 1;
  }
  static std::mutex mu;
  static std::map<std::pair<int, int>, void*> cache;
  std::lock_guard<std::mutex> lk(mu);
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if (precision == AHOC_MIXED) {
    auto key = std::make_pair(N, 4);
    DstTables<float>* tb = (DstTables<float>*)cache[key];
    if (!tb) {
      tb = new DstTables<float>();
      if ((rc = dst_tables_init<float>(*tb, N))) { delete tb; return (ahoc_status)rc; }
      cache[key] = tb;
    }
    rc = dst_pass<float>(*tb, (const float*)in, (float*)out, outer, inner, ni[0], nullptr, 0, st);
  } else if (precision == AHOC_FP64) {
    auto key = std::make_pair(N, 8);
    DstTables<double>* tb = (DstTables<double>*)cache[key];
    if (!tb) {
      tb = new DstTables<double>();
      if ((rc = dst_tables_init<double>(*tb, N))) { delete tb; return (ahoc_status)rc; }
      cache[key] = tb;
    }
    rc = dst_pass<double>(*tb, (const double*)in, (double*)out, outer, inner, ni[0], nullptr, 0, st);
  } else {
    return AHOC_E_INVALID;
  }
  return (ahoc_status)rc;
}

}  // extern "C"
