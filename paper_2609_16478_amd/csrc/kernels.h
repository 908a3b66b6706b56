// Host-side launchers of the stencil, setup and Krylov kernels.
#pragma once

#include "common.h"

namespace ahoc {

// stencil.hip -------------------------------------------------------------------------
template <typename T>
int lift(const Geom& g, const Weights& w, const T* Q, const T* src, T* G, hipStream_t st);
template <typename T>
int rhs_u(const Geom& g, const Weights& w, const T* V, const T* Q, const T* ia, const T* src, T* G,
          hipStream_t st);
template <typename T>
int gather(const Geom& g, const Weights& w, const T* U, const T* Q, const T* af, const T* srcq,
           double* R, hipStream_t st);
// face layers of the homogeneous lift (input of the spectral lift); fixed-order sums of partials
template <typename T>
int face_lift(const Geom& g, const Weights& w, const T* Q, T* Lx, T* Ly, T* Lz, hipStream_t st);
// 3-D: the V-solve's lift layers (weights wv, layouts of face_lift) and the U-solve's
// layers mq Q_b (mq = m1 / alpha_b in Q layout, layouts of face_lift_m) in one tiled pass
// over Q
template <typename T> struct FaceLiftW {
  T w0[3], wf[3], ws[3];  // per face axis: normal, faster and slower tangential couplings
};
template <typename T>
int face_lifts3(const Geom& g, const Weights& wv, const T* Q, const T* mq, T* Lx, T* Ly, T* Lz, T* Ux, T* Uy,
                T* Uz, hipStream_t st);
// out[q] = s * nodal(boundary node of q): a nodal field in Q layout
template <typename T>
int nodal_to_q(const Geom& g, double s, const T* nodal, T* out, hipStream_t st);
// face layers m1 Q_b / alpha_b of the U-solve's source (spectral M), layouts as face_lift
// except the 3-D y faces, [2][n_x'][n_z'] (z fastest)
template <typename T>
int face_lift_m(const Geom& g, const Weights& w, const T* Q, const T* ia, T* Lx, T* Ly, T* Lz, hipStream_t st);
template <typename T>
int partial_sum(long long n, int count, long long stride, const T* in, T* out, hipStream_t st);
// boundary-symbol preconditioner (precond.hip): inverse 2x2 block coefficients per face
// mode from per-axis FP64 tables {s, cos, sin, w_lo} x 3 axes, and their application to
// face spectra of a Q-layout vector
// (tri: the triharmonic chain and q-row; tabs then hold its fourth-derivative combination
// a_1 sin(pi k/N) + ... + a_4 sin(4 pi k/N) in place of w_lo)
int precond_symbol(const Geom& g, const Weights& w, double c, int navier, const double* const* tabs, double* pc,
                   double* qc, hipStream_t st, bool tri = false);
template <typename T>
int precond_modes(const Geom& g, const T* pc, const T* qc, T* x, hipStream_t st);
// boundary residual from face sums formed in spectral space
template <typename T>
int gather_faces(const Geom& g, const T* Fx, const T* Fy, const T* Fz, const T* Q, const T* af,
                 const T* srcq, double* R, hipStream_t st);
template <typename T>
int resid64(const Geom& g, const Weights& w, const double* U, const double* V, const double* Q,
            const double* ia, const double* af, const double* src_u, const double* src_v,
            const double* src_q, T* ru, T* rv, T* rq, hipStream_t st);
int setup_inv_alpha(long long n, const double* alpha, double* ia64, float* ia32, double* bmin,
                    int nb, hipStream_t st);
int setup_face_alpha(const Geom& g, const double* alpha, double* af64, float* af32, hipStream_t st);
// variable shift c (nodal): y = -L_h[V] + M(c V) - src on the interior of a single problem
// (3-D with Q and src null: tiled, and y's row padding is left as it is)
int vapply(const Geom& g, const Weights& w, const double* X, const double* Q, const double* c, const double* src,
           double* y, hipStream_t st);
// per-block min and max (part[2 b], part[2 b + 1]) of n doubles
int minmax_partial(long long n, const double* x, double* part, int nblocks, hipStream_t st);
// Navier faces (the same on every instance of a batch): af = 0 and src_q = -alpha g_L on
// their q-rows
int setup_navier(const Geom& g, int mask, const double* alpha, const double* gL, double* af64, float* af32,
                 double* src_q, hipStream_t st);
// triharmonic extension: interior sources of the W-, V- and U-solves, the q-rows' known part
// and face coefficient, and the boundary residual R = af h^-4 sum a_k U_k - Q - src_q
int tri_sources(const Geom& g, const Weights& w, const double* f, const double* gD, const double* lapu,
                const double* bilap, double* sw, double* sv, double* su, hipStream_t st);
int tri_srcq(const Geom& g, int mask, const double* gD, const double* gN, const double* gNN, const double* tang4,
             const double* bilap, double* src_q, double* af64, float* af32, hipStream_t st);
template <typename T>
int gather_tri(const Geom& g, const T* U, const T* Q, const T* af, const T* srcq, double* R, hipStream_t st);
int setup_sources(const Geom& g, const Weights& w, const double* f, const double* alpha,
                  const double* gD, const double* gN, const double* lapgD, double* src_v,
                  double* src_u, double* src_q, hipStream_t st);
template <typename T>
int out_u(const Geom& g, const T* Ui, const double* gD, double* u, hipStream_t st);
template <typename T>
int out_v(const Geom& g, const T* Vi, const double* Q, const double* vedge, double* v, hipStream_t st);
int mul(long long n, const double* a, const double* b, double* out, hipStream_t st);
template <typename Ti, typename To>
int pitch_copy(long long rows, int cols, const Ti* in, long long ip, To* out, long long op, hipStream_t st);
template <typename Ti, typename To> int convert(long long n, const Ti* in, To* out, hipStream_t st);
template <typename Tx> int accumulate(long long n, const Tx* x, double* y, hipStream_t st);
template <typename Tx>
int absmax_partial(long long n, const Tx* x, double* bmax, int nb, hipStream_t st);
int fill(long long n, double v, double* x, hipStream_t st);

// krylov.hip --------------------------------------------------------------------------
// partial dot products of nvec basis vectors (row stride ld) with w: part[v * nb + b]
int mdot_partial(const double* V, long long ld, int nvec, const double* w, long long n, int ns, double* part,
                 int nbk, hipStream_t st);
int mdot_reduce(const double* part, int nbk, int nvec, int ns, double* out, int ostride, int accumulate,
                hipStream_t st);
// out[s * ostride + v] = <V_v, w> over segment s: partial sums over nbk blocks and their
// reduction, or with nbk == 1 the one block's sums written directly
int mdot(const double* V, long long ld, int nvec, const double* w, long long n, int ns, double* part, int nbk,
         double* out, int ostride, hipStream_t st);
int maxpy(double* w, const double* V, long long ld, int nvec, const double* coef, int cstride, double sign,
          long long n, int ns, hipStream_t st);
int givens_step(int ns, double* H, int m, const double* h1, const double* h2, const double* nrm2, double* cs,
                double* sn, double* gv, int j, double* resid, hipStream_t st);
int axpby(long long n, double a, const double* x, double b, double* y, hipStream_t st);
// y += a x with the per-work-group partial sums of <u, y> (u null: 0) and <y, y>, in part[0..nbk)
// and part[nbk..2 nbk) (reduce with mdot_reduce, nvec 2)
int axpy_dot2(long long n, double a, const double* x, double* y, const double* u, double* part, int nbk,
              hipStream_t st);
// w = a x + b y + c w
int lin3(long long n, double a, const double* x, double b, const double* y, double c, double* w, hipStream_t st);
int scale_by_inv(double* w, long long n, int ns, const double* s, const int* act, hipStream_t st);
// Segment-wise batch utilities (grid.y = segment): x_s = 0 where keep[s] == 0; gather of
// per-instance arrays (device table of device pointers, null = zeros); scatter to them.
int zero_masked(double* x, long long n, int ns, const int* keep, hipStream_t st);
int gather_ptrs(const double* const* src, long long n, int ns, double* out, hipStream_t st);
int scatter_ptrs(const double* in, long long n, int ns, double* const* dst, hipStream_t st);
int back_solve(int ns, const double* H, int m, const double* gv, const int* kk, int kmax, double* y,
               hipStream_t st);
// device-side convergence bookkeeping of Arnoldi step j (see krylov.hip); ist = [act | kk |
// nit | flag | hcnt], ns ints each; hist: 16 doubles per instance; eres: last active estimate
int step_update(int ns, int j, const double* resid, const double* bnorm, double tol, int max_iters, bool inexact,
                int* ist, double* hist, double* eres, hipStream_t st);
// givens_step and step_update in one launch
int givens_update(int ns, double* H, int m, const double* h1, const double* h2, const double* nrm2, double* cs,
                  double* sn, double* gv, int j, double* resid, const double* bnorm, double tol, int max_iters,
                  bool inexact, int* ist, double* hist, double* eres, hipStream_t st);
int fill_int(int* p, long long n, int v, hipStream_t st);
int start_cycle(double* v0, const double* r, long long n, int ns, const double* nrm2, double* gv, int m,
                double* beta, hipStream_t st);

}  // namespace ahoc
