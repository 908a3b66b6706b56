// Boundary-symbol preconditioner of the Schur system (gfx950).
//
// GMRES on S_h Q = b is preconditioned from the right by the inverse of the Schur
// complement of the constant-coefficient problem (alpha = 1) restricted to each pair of
// opposite faces.  With Q a pure sine mode phi(k_b, k_c) on the low face of axis a
// (tangential axes b, c), every step of the matrix-vector product is diagonal in the
// 3-D sine basis, so the response on the two faces normal to a is the same mode times
//   F(k_b, k_c) = h_a^-2 (2/N_a) sum_{k_a} w(k_a) sin(pi k_a/N_a) (m1 - mu T / lambda) / lambda
// with
//   lambda(k)  the eigenvalue of the compact L_h (Dirichlet),
//   mu(k)      the eigenvalue of M = m0 + m1 (face neighbours),
//   T(k_b,k_c) the tangential stencil coupling a face node to the adjacent interior
//              layer (the lift), and m1 sin(pi k_a/N_a) the face value seen by M,
//   w(k_a)     the one-sided combination 6 u_1 - 3/2 u_2 + 2/9 u_3 of mode k_a at the low
//              face (w_lo) or the high face (w_hi = (-1)^(k_a+1) w_lo).
// With beta != 0 (constant alpha) the V-solve divides by lambda - c mu (c = beta/alpha) and
// its lift's normal weight is lowered by c m1, so the term reads (m1 - mu T'/(lambda - c mu)) /
// lambda with T' the shifted lift symbol.
// The triharmonic extension (Sec. 4.2) has constant coefficients; its chain is W from Q
// (the lift, as the V-solve above), V = L^-1 M W (the U-solve above) and U = L^-1 M V, closed
// by the fourth-derivative q-row: the same mode gives
//   F(k_b, k_c) = h_a^-4 (2/N_a) sum_{k_a} w4(k_a) sin(pi k_a/N_a) mu (m1 - mu T / lambda) / lambda^2
// with w4 the row's combination a_1 u_1 + ... + a_4 u_4 of mode k_a.
// Low-low gives sigma = F_lo - 1 (the -Q of the residual), low-high gives tau = F_hi;
// by symmetry the 2x2 block per mode is [[sigma, tau], [tau, sigma]].  A Navier face's rows
// are alpha g_L - Q, so its row of the block is (0, -1) (the opposite face's row keeps
// sigma, tau): the block becomes triangular, or -I with both faces Navier.  Applying the
// preconditioner is a 2-D DST of every face array, one 2x2 solve per mode and pair,
// and the inverse 2-D DST: O(N^(d-1) log N), negligible next to a matvec.
#include "common.h"
#include "kernels.h"

namespace ahoc {

namespace {

constexpr int TPB = 256;

inline unsigned nblk(long long n) {
  long long b = (n + TPB - 1) / TPB;
  if (b > 1048576) b = 1048576;
  return (unsigned)(b < 1 ? 1 : b);
}

// Per-axis FP64 tables for k = 1..N_a-1 (index k-1): s(k) = -(4/h^2) sin^2(pi k / 2N),
// cos(pi k / N), sin(pi k / N), w_lo(k).
struct AxisTab {
  const double* s;
  const double* c;
  const double* sn;
  const double* wl;
};

struct SymArgs {
  Geom g;
  Weights w;   // the lift stencil of the v-equation (with the shift in its normal weight)
  double c;    // the v-equation's shift beta/alpha (0 for beta = 0)
  int navier;  // bit f set: face f (2 axis + side) is a Navier face
  int tri;     // 1: the triharmonic chain (one more solve, h^-4 fourth-derivative row)
  AxisTab t[3];
  // the inverse 2x2 block [[a, b], [c, d]] of a mode (rows and columns: low face, high
  // face) is stored at the mode's low entry lo and high entry hi as
  // pc[lo] = a, qc[lo] = b, qc[hi] = c, pc[hi] = d
  double* pc;
  double* qc;
};

__device__ __forceinline__ int pair_ce(int a, int b) {
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  return (lo == 0 && hi == 1) ? 0 : (lo == 0 ? 1 : 2);
}

// One thread per low-face entry (mode) of every axis.
template <int DIM>
__global__ void k_symbol(SymArgs A) {
  const Geom& g = A.g;
  long long tot = 0;
  for (int a = 0; a < DIM; ++a) tot += g.face_off[2 * a + 1] - g.face_off[2 * a];
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    int a = 0;
    long long t = e;
    while (t >= g.face_off[2 * a + 1] - g.face_off[2 * a]) {
      t -= g.face_off[2 * a + 1] - g.face_off[2 * a];
      ++a;
    }
    // tangential axes b (fastest in the face layout) and c
    int b, c = -1;
    if (DIM == 2) {
      b = 1 - a;
    } else {
      b = a == 0 ? 1 : 0;
      c = a == 2 ? 1 : 2;
    }
    const int kb = (int)(DIM == 3 ? t % g.ni[b] : t);  // k_b - 1
    const int kc = DIM == 3 ? (int)(t / g.ni[b]) : 0;  // k_c - 1
    const double sb = A.t[b].s[kb], cb = A.t[b].c[kb];
    const double sc = DIM == 3 ? A.t[c].s[kc] : 0.0, cc = DIM == 3 ? A.t[c].c[kc] : 0.0;
    const double ha2 = g.h[a] * g.h[a], hb2 = g.h[b] * g.h[b];
    const double hc2 = DIM == 3 ? g.h[c] * g.h[c] : 0.0;
    const double cab = (ha2 + hb2) / 12.0, cac = (ha2 + hc2) / 12.0, cbc = (hb2 + hc2) / 12.0;
    // lift stencil of the face, tangential symbol
    double T = A.w.cf[a] + 2.0 * A.w.ce[DIM == 3 ? pair_ce(a, b) : 0] * cb;
    if (DIM == 3) T += 2.0 * A.w.ce[pair_ce(a, c)] * cc;
    const double mt = A.w.m0 + 2.0 * A.w.m1 * (cb + (DIM == 3 ? cc : 0.0));
    double sig = 0, tau = 0;
    const int na = g.ni[a];
    for (int k = 0; k < na; ++k) {
      const double sa = A.t[a].s[k];
      const double lam = sa + sb + sc + cab * sa * sb + cac * sa * sc + cbc * sb * sc;
      const double mu = mt + 2.0 * A.w.m1 * A.t[a].c[k];
      // V-solve with the shifted eigenvalue lambda - c mu, U-solve with lambda (the
      // triharmonic chain: one more solve with M, mu / lambda)
      double term = A.t[a].sn[k] * (A.w.m1 - mu * T / (lam - A.c * mu)) / lam;
      if (A.tri) term *= mu / lam;
      const double wl = A.t[a].wl[k];
      sig += wl * term;
      tau += ((k & 1) ? -wl : wl) * term;  // w_hi(k) = (-1)^(k+1) w_lo(k), k = index + 1
    }
    const double f = A.tri ? 2.0 / (ha2 * ha2 * g.n[a]) : 2.0 / (ha2 * g.n[a]);
    sig = f * sig - 1.0;
    tau = f * tau;
    double norm = 2.0 / g.n[b];
    if (DIM == 3) norm *= 2.0 / g.n[c];
    const long long lo = g.face_off[2 * a] + t, hi = g.face_off[2 * a + 1] + t;
    const bool nl = (A.navier >> (2 * a)) & 1, nh = (A.navier >> (2 * a + 1)) & 1;
    double ia, ib, ic, id;  // inverse of the block
    if (!nl && !nh) {  // [[sig, tau], [tau, sig]]
      const double det = sig * sig - tau * tau;
      ia = id = sig / det;
      ib = ic = -tau / det;
    } else if (nl && nh) {  // -I
      ia = id = -1.0;
      ib = ic = 0.0;
    } else if (nh) {  // [[sig, tau], [0, -1]]
      ia = 1.0 / sig;
      ib = tau / sig;
      ic = 0.0;
      id = -1.0;
    } else {  // [[-1, 0], [tau, sig]]
      ia = -1.0;
      ib = 0.0;
      ic = tau / sig;
      id = 1.0 / sig;
    }
    A.pc[lo] = norm * ia;
    A.qc[lo] = norm * ib;
    A.qc[hi] = norm * ic;
    A.pc[hi] = norm * id;
  }
}

// In place on face spectra: (lo, hi) <- (pc[lo] lo + qc[lo] hi, qc[hi] lo + pc[hi] hi) for
// every low-face entry of every instance (the coefficients are shared by the instances of a
// batch).
template <typename T, int DIM>
__global__ void k_modes(Geom g, const T* __restrict__ pc, const T* __restrict__ qc, T* __restrict__ x) {
  x += (long long)blockIdx.y * g.nq;  // instance of a batch (gridDim.y = g.nb)
  long long tot = 0;
  for (int a = 0; a < DIM; ++a) tot += g.face_off[2 * a + 1] - g.face_off[2 * a];
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    int a = 0;
    long long t = e;
    while (t >= g.face_off[2 * a + 1] - g.face_off[2 * a]) {
      t -= g.face_off[2 * a + 1] - g.face_off[2 * a];
      ++a;
    }
    const long long lo = g.face_off[2 * a] + t, hi = g.face_off[2 * a + 1] + t;
    const T xl = x[lo], xh = x[hi];
    x[lo] = pc[lo] * xl + qc[lo] * xh;
    x[hi] = qc[hi] * xl + pc[hi] * xh;
  }
}

}  // namespace

int precond_symbol(const Geom& g, const Weights& w, double c, int navier, const double* const* tabs, double* pc,
                   double* qc, hipStream_t st, bool tri) {
  SymArgs A;
  A.g = g;
  A.w = w;
  A.c = c;
  A.navier = navier;
  A.tri = tri ? 1 : 0;
  for (int a = 0; a < 3; ++a) {
    A.t[a].s = tabs[4 * a];
    A.t[a].c = tabs[4 * a + 1];
    A.t[a].sn = tabs[4 * a + 2];
    A.t[a].wl = tabs[4 * a + 3];
  }
  A.pc = pc;
  A.qc = qc;
  const long long tot = g.nq / 2;
  if (g.dim == 3) hipLaunchKernelGGL((k_symbol<3>), dim3(nblk(tot)), dim3(TPB), 0, st, A);
  else hipLaunchKernelGGL((k_symbol<2>), dim3(nblk(tot)), dim3(TPB), 0, st, A);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

template <typename T>
int precond_modes(const Geom& g, const T* pc, const T* qc, T* x, hipStream_t st) {
  const long long tot = g.nq / 2;
  if (g.dim == 3) hipLaunchKernelGGL((k_modes<T, 3>), dim3(nblk(tot), g.nb), dim3(TPB), 0, st, g, pc, qc, x);
  else hipLaunchKernelGGL((k_modes<T, 2>), dim3(nblk(tot), g.nb), dim3(TPB), 0, st, g, pc, qc, x);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

template int precond_modes<float>(const Geom&, const float*, const float*, float*, hipStream_t);
template int precond_modes<double>(const Geom&, const double*, const double*, double*, hipStream_t);

}  // namespace ahoc
