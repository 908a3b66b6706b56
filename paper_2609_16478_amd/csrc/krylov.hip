// FP64 Krylov kernels of the device-resident GMRES(m) (matrix-free GMRES on
// S_h Q = b, Sec. 2.3).  Arnoldi uses classical Gram-Schmidt with one
// re-orthogonalisation (two block dot-product sweeps instead of j dependent
// ones), Givens rotations keep the least-squares residual |g_{j+1}|.
// Reductions are two-stage with a fixed order, so results are reproducible.
#include "common.h"
#include "kernels.h"

namespace ahoc {

namespace {

constexpr int TPB = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Every kernel works on `ns` independent segments (the instances of a batch, 1 for a
// single problem): a vector of the Krylov basis is ns consecutive segments of length n,
// and each segment has its own dot products, Hessenberg matrix, rotations and norms.
// Per-segment small arrays: H [ns][m][m+1] (column j at j*(m+1)), cs, sn [ns][m],
// gv, y, h1, h2 [ns][m+1], nrm, resid [ns][2], beta [ns], act [ns].

// part[(s * nvec + v) * gridDim.x + block] = partial sum of <V_v, w> over segment s, or with
// one block per segment and `out` given, the sum itself at out[s * ostride + v].  The
// vectors are taken MDC at a time, so that w is read once per group of vectors rather than
// once per vector; each vector's sum runs over the same elements in the same order either way.
constexpr int MDC = 8;
// The group's MDC sums are reduced together: across each wavefront with shuffles, then the
// TPB/64 wavefront sums added in wavefront order by one thread per vector (one barrier per
// group; the LDS rows alternate between groups, so a group's rows are not overwritten before
// they are read).
__global__ void k_mdot_partial(const double* __restrict__ V, long long ld, int nvec,
                               const double* __restrict__ w, long long n, double* __restrict__ part,
                               double* __restrict__ out, int ostride) {
  constexpr int NW = TPB / 64;
  __shared__ double red[2][NW][MDC];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long long s0 = blockIdx.y * n;
  const double* ws = w + s0;
  for (int v0 = 0; v0 < nvec; v0 += MDC) {
    const int nv = nvec - v0 < MDC ? nvec - v0 : MDC;
    double acc[MDC];
#pragma unroll
    for (int c = 0; c < MDC; ++c) acc[c] = 0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
      const double we = ws[e];
#pragma unroll
      for (int c = 0; c < MDC; ++c)
        if (c < nv) acc[c] += V[(long long)(v0 + c) * ld + s0 + e] * we;
    }
#pragma unroll
    for (int c = 0; c < MDC; ++c) {
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) acc[c] += __shfl_xor(acc[c], m, 64);
    }
    const int buf = (v0 / MDC) & 1;
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < MDC; ++c) red[buf][wv][c] = acc[c];
    }
    __syncthreads();
    if (threadIdx.x < nv) {
      const int c = threadIdx.x;
      double r = red[buf][0][c];
#pragma unroll
      for (int k = 1; k < NW; ++k) r += red[buf][k][c];
      if (out) out[(long long)blockIdx.y * ostride + v0 + c] = r;
      else part[((long long)blockIdx.y * nvec + v0 + c) * gridDim.x + blockIdx.x] = r;
    }
  }
}

// out[s * ostride + v] (+)= sum of the partials of (segment s, vector v)
__global__ void k_mdot_reduce(const double* __restrict__ part, int nbk, int nvec, double* __restrict__ out,
                              int ostride, int accumulate) {
  __shared__ double red[TPB];
  const int v = blockIdx.x;
  const long long sg = blockIdx.y;
  double acc = 0;
  for (int b = threadIdx.x; b < nbk; b += blockDim.x) acc += part[(sg * nvec + v) * nbk + b];
  const double r = block_sum(acc, red);
  if (threadIdx.x == 0) {
    double* o = out + sg * ostride + v;
    *o = accumulate ? *o + r : r;
  }
}

// w_s += sign * sum_v coef[s * cstride + v] V_v  on each segment s
__global__ void k_maxpy(double* __restrict__ w, const double* __restrict__ V, long long ld, int nvec,
                        const double* __restrict__ coef, int cstride, double sign, long long n) {
  const long long s0 = blockIdx.y * n;
  const double* c = coef + (long long)blockIdx.y * cstride;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    double acc = 0;
    for (int v = 0; v < nvec; ++v) acc += c[v] * V[(long long)v * ld + s0 + e];
    w[s0 + e] += sign * acc;
  }
}

// one thread per segment
__device__ __forceinline__ void givens_body(int sg, double* H, int m, const double* h1, const double* h2,
                                            const double* nrm2, double* cs, double* sn, double* gv, int j,
                                            double* resid) {
  const int ldh = m + 1;
  double* col = H + (long long)sg * m * ldh + (long long)j * ldh;
  const double* a1 = h1 + (long long)sg * ldh;
  const double* a2 = h2 + (long long)sg * ldh;
  double* c_ = cs + (long long)sg * m;
  double* s_ = sn + (long long)sg * m;
  double* g_ = gv + (long long)sg * ldh;
  const double nn = sqrt(fmax(nrm2[2 * sg], 0.0));
  for (int i = 0; i <= j; ++i) col[i] = a1[i] + a2[i];
  col[j + 1] = nn;
  for (int i = 0; i < j; ++i) {
    const double t = c_[i] * col[i] + s_[i] * col[i + 1];
    col[i + 1] = -s_[i] * col[i] + c_[i] * col[i + 1];
    col[i] = t;
  }
  const double a = col[j], b = col[j + 1];
  const double rho = hypot(a, b);
  const double c = rho > 0 ? a / rho : 1.0, s = rho > 0 ? b / rho : 0.0;
  c_[j] = c;
  s_[j] = s;
  col[j] = rho;
  g_[j + 1] = -s * g_[j];
  g_[j] = c * g_[j];
  resid[2 * sg] = fabs(g_[j + 1]);
  // keep the un-rotated subdiagonal for normalising v_{j+1}
  resid[2 * sg + 1] = nn;
  col[j + 1] = 0.0;
}

__global__ void k_givens(int ns, double* H, int m, const double* h1, const double* h2, const double* nrm2,
                         double* cs, double* sn, double* gv, int j, double* resid) {
  const int sg = blockIdx.x * blockDim.x + threadIdx.x;
  if (sg >= ns) return;
  givens_body(sg, H, m, h1, h2, nrm2, cs, sn, gv, j, resid);
}

__global__ void k_axpby(long long n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    y[e] = b == 0.0 ? a * x[e] : a * x[e] + b * y[e];
}

// y += a x, with the partial sums of <u, y> (u may be null: 0) and <y, y> of the updated y:
// part[b] and part[gridDim.x + b] for work-group b
__global__ void k_axpy_dot2(long long n, double a, const double* __restrict__ x, double* __restrict__ y,
                            const double* __restrict__ u, double* __restrict__ part) {
  __shared__ double red[TPB];
  double su = 0, sy = 0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const double v = y[e] + a * x[e];
    y[e] = v;
    if (u) su += u[e] * v;
    sy += v * v;
  }
  const double r0 = block_sum(su, red);
  const double r1 = block_sum(sy, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = r0;
    part[gridDim.x + blockIdx.x] = r1;
  }
}

// w = a x + b y + c w
__global__ void k_lin3(long long n, double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                       double c, double* __restrict__ w) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    w[e] = a * x[e] + b * y[e] + c * w[e];
}

// w_s *= 1 / resid[s][1]; segments that are no longer active (or have a zero norm) get 0,
// so a converged instance continues with zero basis vectors
__global__ void k_scale_inv(double* __restrict__ w, long long n, const double* __restrict__ s,
                            const int* __restrict__ act) {
  const double d = s[2 * blockIdx.y + 1];
  const double r = (d > 0 && (!act || act[blockIdx.y])) ? 1.0 / d : 0.0;
  const long long s0 = blockIdx.y * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    w[s0 + e] *= r;
}

// x_s = 0 on every segment s with keep[s] == 0
__global__ void k_zero_masked(double* __restrict__ x, long long n, const int* __restrict__ keep) {
  if (keep[blockIdx.y]) return;
  const long long s0 = blockIdx.y * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    x[s0 + e] = 0.0;
}

// out_s = src[s] (or 0 where src[s] is null): concatenate per-instance arrays of length n
__global__ void k_gather_ptrs(const double* const* __restrict__ src, long long n, double* __restrict__ out) {
  const double* p = src[blockIdx.y];
  double* o = out + blockIdx.y * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    o[e] = p ? p[e] : 0.0;
}

// dst[s] = in_s: split a batch array into per-instance arrays of length n
__global__ void k_scatter_ptrs(const double* __restrict__ in, long long n, double* const* __restrict__ dst) {
  double* p = dst[blockIdx.y];
  const double* x = in + blockIdx.y * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    p[e] = x[e];
}

// one thread per segment: y_s[0..k_s) from the rotated triangle, y_s[k_s..kmax) = 0
__global__ void k_back_solve(int ns, const double* H, int m, const double* gv, const int* kk, int kmax, double* y) {
  const int sg = blockIdx.x * blockDim.x + threadIdx.x;
  if (sg >= ns) return;
  const int ldh = m + 1;
  const double* Hs = H + (long long)sg * m * ldh;
  const double* g_ = gv + (long long)sg * ldh;
  double* ys = y + (long long)sg * ldh;
  const int k = kk[sg];
  for (int i = k; i < kmax; ++i) ys[i] = 0.0;
  for (int i = k - 1; i >= 0; --i) {
    double t = g_[i];
    for (int c = i + 1; c < k; ++c) t -= Hs[(long long)c * ldh + i] * ys[c];
    ys[i] = t / Hs[(long long)i * ldh + i];
  }
}

__global__ void k_start(double* __restrict__ v0, const double* __restrict__ r, long long n,
                        const double* __restrict__ nrm2, double* gv, int m, double* beta) {
  const long long sg = blockIdx.y;
  const double b = sqrt(fmax(nrm2[2 * sg], 0.0));
  const double ib = b > 0 ? 1.0 / b : 0.0;
  const long long s0 = sg * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    v0[s0 + e] = r[s0 + e] * ib;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double* g_ = gv + sg * (m + 1);
    g_[0] = b;
    for (int i = 1; i <= m; ++i) g_[i] = 0.0;
    beta[sg] = b;
  }
}

// Per-instance bookkeeping after the Givens update of Arnoldi step j, on the device, so
// that the host need not read the residual estimates every step.  ist = [act | kk | nit |
// flag | hcnt] (ns ints each): an active instance counts the step, records its Krylov
// dimension j + 1 and stops -- flag 1 -- when |g_{j+1}| <= tol ||b||, with flag 2 when the
// estimate is not finite or, for an FP32 operator (inexact), when eight steps gained less
// than a factor 2 below 1e-2 (ring of its last 16 estimates in hist), and without a flag at
// the iteration cap.  eres keeps each instance's estimate of its last active step.
__device__ __forceinline__ void update_body(int s, int ns, int j, const double* resid, const double* bnorm,
                                            double tol, int max_iters, int inexact, int* ist, double* hist,
                                            double* eres) {
  int* act = ist;
  int* kk = ist + ns;
  int* nit = ist + 2 * ns;
  int* flag = ist + 3 * ns;
  int* hcnt = ist + 4 * ns;
  if (!act[s]) return;
  const int it = ++nit[s];
  kk[s] = j + 1;
  const double est = resid[2 * s] / bnorm[s];
  eres[s] = est;
  bool stop = false;
  if (!isfinite(est)) {
    flag[s] = 2;
    stop = true;
  } else if (est <= tol) {
    flag[s] = 1;
    stop = true;
  } else {
    if (inexact) {
      double* hs = hist + 16LL * s;
      const int hc = hcnt[s] + 1;
      hs[(hc - 1) & 15] = est;
      hcnt[s] = hc;
      if (hc > 8 && est < 1e-2 && est > 0.5 * hs[(hc - 9) & 15]) {
        flag[s] = 2;
        stop = true;
      }
    }
    if (it >= max_iters) stop = true;
  }
  if (stop) act[s] = 0;
}

__global__ void k_step_update(int ns, int j, const double* __restrict__ resid, const double* __restrict__ bnorm,
                              double tol, int max_iters, int inexact, int* __restrict__ ist,
                              double* __restrict__ hist, double* __restrict__ eres) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  update_body(s, ns, j, resid, bnorm, tol, max_iters, inexact, ist, hist, eres);
}

// k_givens then k_step_update for each segment, in one launch (each segment's update reads
// only the residual estimate its own rotation wrote)
__global__ void k_givens_update(int ns, double* H, int m, const double* h1, const double* h2, const double* nrm2,
                                double* cs, double* sn, double* gv, int j, double* resid, const double* bnorm,
                                double tol, int max_iters, int inexact, int* ist, double* hist, double* eres) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  givens_body(s, H, m, h1, h2, nrm2, cs, sn, gv, j, resid);
  update_body(s, ns, j, resid, bnorm, tol, max_iters, inexact, ist, hist, eres);
}

__global__ void k_fill_int(int* __restrict__ p, long long n, int v) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    p[e] = v;
}

inline unsigned nblk(long long n, int cap) {
  long long b = (n + TPB - 1) / TPB;
  if (b > cap) b = cap;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

int mdot_partial(const double* V, long long ld, int nvec, const double* w, long long n, int ns, double* part,
                 int nbk, hipStream_t st) {
  hipLaunchKernelGGL(k_mdot_partial, dim3(nbk, ns), dim3(TPB), 0, st, V, ld, nvec, w, n, part, nullptr, 0);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int mdot(const double* V, long long ld, int nvec, const double* w, long long n, int ns, double* part, int nbk,
         double* out, int ostride, hipStream_t st) {
  if (nbk == 1) {  // one block per segment: its sum is the result (no reduction launch)
    hipLaunchKernelGGL(k_mdot_partial, dim3(1, ns), dim3(TPB), 0, st, V, ld, nvec, w, n, part, out, ostride);
    AHOC_HIP_TRY(hipGetLastError());
    return ST_OK;
  }
  TRY_ST(mdot_partial(V, ld, nvec, w, n, ns, part, nbk, st));
  return mdot_reduce(part, nbk, nvec, ns, out, ostride, 0, st);
}

int mdot_reduce(const double* part, int nbk, int nvec, int ns, double* out, int ostride, int accumulate,
                hipStream_t st) {
  hipLaunchKernelGGL(k_mdot_reduce, dim3(nvec, ns), dim3(TPB), 0, st, part, nbk, nvec, out, ostride, accumulate);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int maxpy(double* w, const double* V, long long ld, int nvec, const double* coef, int cstride, double sign,
          long long n, int ns, hipStream_t st) {
  hipLaunchKernelGGL(k_maxpy, dim3(nblk(n, 65536), ns), dim3(TPB), 0, st, w, V, ld, nvec, coef, cstride, sign, n);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int givens_step(int ns, double* H, int m, const double* h1, const double* h2, const double* nrm2, double* cs,
                double* sn, double* gv, int j, double* resid, hipStream_t st) {
  hipLaunchKernelGGL(k_givens, dim3((ns + 63) / 64), dim3(64), 0, st, ns, H, m, h1, h2, nrm2, cs, sn, gv, j, resid);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int axpby(long long n, double a, const double* x, double b, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3(nblk(n, 65536)), dim3(TPB), 0, st, n, a, x, b, y);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int axpy_dot2(long long n, double a, const double* x, double* y, const double* u, double* part, int nbk,
              hipStream_t st) {
  hipLaunchKernelGGL(k_axpy_dot2, dim3(nbk), dim3(TPB), 0, st, n, a, x, y, u, part);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int lin3(long long n, double a, const double* x, double b, const double* y, double c, double* w, hipStream_t st) {
  hipLaunchKernelGGL(k_lin3, dim3(nblk(n, 65536)), dim3(TPB), 0, st, n, a, x, b, y, c, w);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int scale_by_inv(double* w, long long n, int ns, const double* s, const int* act, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_inv, dim3(nblk(n, 65536), ns), dim3(TPB), 0, st, w, n, s, act);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int zero_masked(double* x, long long n, int ns, const int* keep, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_masked, dim3(nblk(n, 65536), ns), dim3(TPB), 0, st, x, n, keep);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int gather_ptrs(const double* const* src, long long n, int ns, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_ptrs, dim3(nblk(n, 65536), ns), dim3(TPB), 0, st, src, n, out);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int scatter_ptrs(const double* in, long long n, int ns, double* const* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter_ptrs, dim3(nblk(n, 65536), ns), dim3(TPB), 0, st, in, n, dst);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int back_solve(int ns, const double* H, int m, const double* gv, const int* kk, int kmax, double* y,
               hipStream_t st) {
  hipLaunchKernelGGL(k_back_solve, dim3((ns + 63) / 64), dim3(64), 0, st, ns, H, m, gv, kk, kmax, y);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int step_update(int ns, int j, const double* resid, const double* bnorm, double tol, int max_iters, bool inexact,
                int* ist, double* hist, double* eres, hipStream_t st) {
  hipLaunchKernelGGL(k_step_update, dim3((ns + 63) / 64), dim3(64), 0, st, ns, j, resid, bnorm, tol, max_iters,
                     inexact ? 1 : 0, ist, hist, eres);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int givens_update(int ns, double* H, int m, const double* h1, const double* h2, const double* nrm2, double* cs,
                  double* sn, double* gv, int j, double* resid, const double* bnorm, double tol, int max_iters,
                  bool inexact, int* ist, double* hist, double* eres, hipStream_t st) {
  hipLaunchKernelGGL(k_givens_update, dim3((ns + 63) / 64), dim3(64), 0, st, ns, H, m, h1, h2, nrm2, cs, sn, gv, j,
                     resid, bnorm, tol, max_iters, inexact ? 1 : 0, ist, hist, eres);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int fill_int(int* p, long long n, int v, hipStream_t st) {
  if (n <= 0) return ST_OK;
  hipLaunchKernelGGL(k_fill_int, dim3(nblk(n, 4096)), dim3(TPB), 0, st, p, n, v);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int start_cycle(double* v0, const double* r, long long n, int ns, const double* nrm2, double* gv, int m,
                double* beta, hipStream_t st) {
  hipLaunchKernelGGL(k_start, dim3(nblk(n, 65536), ns), dim3(TPB), 0, st, v0, r, n, nrm2, gv, m, beta);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

}  // namespace ahoc
