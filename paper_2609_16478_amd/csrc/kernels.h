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
template <typename T>
int partial_sum(long long n, int count, long long stride, const T* in, T* out, hipStream_t st);
// boundary-symbol preconditioner (precond.hip): inverse 2x2 block coefficients per face
// mode from per-axis FP64 tables {s, cos, sin, w_lo} x 3 axes, and their application to
// face spectra of a Q-layout vector
int precond_symbol(const Geom& g, const Weights& w, const double* const* tabs, double* pc, double* qc,
                   hipStream_t st);
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
int mdot_partial(const double* V, long long ld, int nvec, const double* w, long long n,
                 double* part, int nb, hipStream_t st);
// out[v] (+)= sum_b part[v * nb + b]
int mdot_reduce(const double* part, int nb, int nvec, double* out, int accumulate, hipStream_t st);
// w += sign * sum_v coef[v] V[v]
int maxpy(double* w, const double* V, long long ld, int nvec, const double* coef, double sign,
          long long n, hipStream_t st);
// Arnoldi column finish + Givens update for column j (single work-item kernel)
int givens_step(double* H, int ldh, const double* h1, const double* h2, const double* nrm2,
                double* cs, double* sn, double* gv, int j, double* resid, hipStream_t st);
// y = a x + b y   (b == 0: y is overwritten without being read)
int axpby(long long n, double a, const double* x, double b, double* y, hipStream_t st);
// w *= 1 / H[j+1, j]  (zero if the norm vanished)
int scale_by_inv(double* w, long long n, const double* s, hipStream_t st);
// y = H(0:k,0:k)^{-1} g(0:k)
int back_solve(const double* H, int ldh, const double* gv, int k, double* y, hipStream_t st);
// v0 = r / ||r||, g = (||r||, 0, ...)
int start_cycle(double* v0, const double* r, long long n, const double* nrm2, double* gv, int m,
                double* beta, hipStream_t st);

}  // namespace ahoc
