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

__global__ void k_mdot_partial(const double* __restrict__ V, long long ld, int nvec,
                               const double* __restrict__ w, long long n, double* __restrict__ part) {
  __shared__ double red[TPB];
  for (int v = 0; v < nvec; ++v) {
    const double* x = V + (long long)v * ld;
    double acc = 0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x)
      acc += x[e] * w[e];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) part[(long long)v * gridDim.x + blockIdx.x] = s;
  }
}

__global__ void k_mdot_reduce(const double* __restrict__ part, int nb, double* __restrict__ out, int accumulate) {
  __shared__ double red[TPB];
  const int v = blockIdx.x;
  double acc = 0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += part[(long long)v * nb + b];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) out[v] = accumulate ? out[v] + s : s;
}

__global__ void k_maxpy(double* __restrict__ w, const double* __restrict__ V, long long ld, int nvec,
                        const double* __restrict__ coef, double sign, long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    double acc = 0;
    for (int v = 0; v < nvec; ++v) acc += coef[v] * V[(long long)v * ld + e];
    w[e] += sign * acc;
  }
}

__global__ void k_givens(double* H, int ldh, const double* h1, const double* h2, const double* nrm2,
                         double* cs, double* sn, double* gv, int j, double* resid) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double* col = H + (long long)j * ldh;
  for (int i = 0; i <= j; ++i) col[i] = h1[i] + h2[i];
  col[j + 1] = sqrt(fmax(nrm2[0], 0.0));
  for (int i = 0; i < j; ++i) {
    const double t = cs[i] * col[i] + sn[i] * col[i + 1];
    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
    col[i] = t;
  }
  const double a = col[j], b = col[j + 1];
  const double rho = hypot(a, b);
  const double c = rho > 0 ? a / rho : 1.0, s = rho > 0 ? b / rho : 0.0;
  cs[j] = c;
  sn[j] = s;
  col[j] = rho;
  gv[j + 1] = -s * gv[j];
  gv[j] = c * gv[j];
  resid[0] = fabs(gv[j + 1]);
  // keep the un-rotated subdiagonal for normalising v_{j+1}
  resid[1] = sqrt(fmax(nrm2[0], 0.0));
  col[j + 1] = 0.0;
}

__global__ void k_axpby(long long n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    y[e] = b == 0.0 ? a * x[e] : a * x[e] + b * y[e];
}

__global__ void k_scale_inv(double* __restrict__ w, long long n, const double* __restrict__ s) {
  const double d = s[1];
  const double r = d > 0 ? 1.0 / d : 0.0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    w[e] *= r;
}

__global__ void k_back_solve(const double* H, int ldh, const double* gv, int k, double* y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    double t = gv[i];
    for (int c = i + 1; c < k; ++c) t -= H[(long long)c * ldh + i] * y[c];
    y[i] = t / H[(long long)i * ldh + i];
  }
}

__global__ void k_start(double* __restrict__ v0, const double* __restrict__ r, long long n,
                        const double* __restrict__ nrm2, double* gv, int m, double* beta) {
  const double b = sqrt(fmax(nrm2[0], 0.0));
  const double ib = b > 0 ? 1.0 / b : 0.0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    v0[e] = r[e] * ib;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    gv[0] = b;
    for (int i = 1; i <= m; ++i) gv[i] = 0.0;
    beta[0] = b;
  }
}

inline unsigned nblk(long long n, int cap) {
  long long b = (n + TPB - 1) / TPB;
  if (b > cap) b = cap;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

int mdot_partial(const double* V, long long ld, int nvec, const double* w, long long n, double* part,
                 int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_mdot_partial, dim3(nb), dim3(TPB), 0, st, V, ld, nvec, w, n, part);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int mdot_reduce(const double* part, int nb, int nvec, double* out, int accumulate, hipStream_t st) {
  hipLaunchKernelGGL(k_mdot_reduce, dim3(nvec), dim3(TPB), 0, st, part, nb, out, accumulate);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int maxpy(double* w, const double* V, long long ld, int nvec, const double* coef, double sign,
          long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_maxpy, dim3(nblk(n, 65536)), dim3(TPB), 0, st, w, V, ld, nvec, coef, sign, n);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int givens_step(double* H, int ldh, const double* h1, const double* h2, const double* nrm2,
                double* cs, double* sn, double* gv, int j, double* resid, hipStream_t st) {
  hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, st, H, ldh, h1, h2, nrm2, cs, sn, gv, j, resid);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int axpby(long long n, double a, const double* x, double b, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3(nblk(n, 65536)), dim3(TPB), 0, st, n, a, x, b, y);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int scale_by_inv(double* w, long long n, const double* s, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_inv, dim3(nblk(n, 65536)), dim3(TPB), 0, st, w, n, s);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int back_solve(const double* H, int ldh, const double* gv, int k, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_back_solve, dim3(1), dim3(64), 0, st, H, ldh, gv, k, y);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

int start_cycle(double* v0, const double* r, long long n, const double* nrm2, double* gv, int m,
                double* beta, hipStream_t st) {
  hipLaunchKernelGGL(k_start, dim3(nblk(n, 65536)), dim3(TPB), 0, st, v0, r, n, nrm2, gv, m, beta);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

}  // namespace ahoc
