// Allocation-free Dirichlet solve (gfx950): ahoc_poisson without a handle.
//
// The fast Poisson solver of Sec. 2.3 / Remark 2 -- w = L_int^{-1} g by sine transforms
// along every axis, the slowest-axis pass dividing by the compact Laplacian's eigenvalue --
// for callers that cannot allocate device memory.  Its work array (the padded interior) and
// the per-axis transform and eigenvalue tables live in one file-scope device array of
// NOALLOC_SCRATCH_BYTES per GPU, held until the process ends.  The tables are generated on
// the device by a small kernel every call (no host-to-device copies), and the passes are the
// same kernels ahoc_poisson launches.
//
// The array's name is a host-side stand-in: host code uses only the device address that
// hipGetSymbolAddress returns for the current device (cached per device).  Calls that
// overlap on one GPU share the array and race.
#include "../../include/ahoc.h"
#include "common.h"
#include "kernels.h"

#include <algorithm>
#include <mutex>

namespace ahoc {

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
constexpr size_t NOALLOC_TABLE_BYTES = (size_t)1 << 20;  // per-axis tables, then the work array
constexpr int NOALLOC_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
void* g_ptr[NOALLOC_MAX_DEVICES] = {nullptr};

// Device address of `scratch` on the current device (looked up once per device).
int scratch_ptr(void** out) {
  int dev = 0;
  AHOC_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
    set_last_error("device index beyond the no-alloc table", "ahoc_poisson_noalloc");
    return ST_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_last_error(hipGetErrorString(e), "hipGetSymbolAddress(scratch)");
      return ST_HIP;
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return ST_OK;
}

// Tables of one axis of length N (N - 1 interior points), spacing h, generated in FP64:
//   plan:   tw[k] = exp(-2 pi i k / N) (k < N), sn[m] = sin(pi m / N) (m <= N/2)
//   direct: sn[j] = sin(pi j / N) over one period (j < 2N)
//   s[k-1] = -(4 / h^2) sin^2(pi k / (2N)), the 1-D second difference on sine mode k
template <typename T>
__global__ void k_axis_tables(int N, int plan, double h, cx<T>* tw, T* sn, T* s) {
  const int nsn = plan ? N / 2 + 1 : 2 * N;
  const int total = (plan ? N : 0) + nsn + (N - 1);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    int i = e;
    if (plan && i < N) {
      double sv, cv;
      sincospi(2.0 * i / N, &sv, &cv);
      tw[i].x = (T)cv;
      tw[i].y = (T)(-sv);
      continue;
    }
    if (plan) i -= N;
    if (i < nsn) {
      sn[i] = (T)sinpi((double)i / N);
      continue;
    }
    i -= nsn;
    const double sv = sinpi((double)(i + 1) / (2.0 * N));
    s[i] = (T)(-4.0 * sv * sv / (h * h));
  }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Dense FP64 interior rows (cols values each) into the padded work array (row pitch px),
// writing the padding columns as zeros: the transform kernels read a row's padding slot with
// a zero weight, so whatever an earlier call left there (a NaN bit pattern included) must not
// survive into this one.
template <typename T>
__global__ void k_load_padded(long long rows, int cols, int px, const double* __restrict__ in, T* __restrict__ out) {
  const long long n = rows * px;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const long long r = e / px;
    const int c = (int)(e - r * px);
    out[e] = c < cols ? (T)in[r * cols + c] : T(0);
  }
}

template <typename T>
int poisson_noalloc(int dim, const int* n, const double* lo, const double* hi, const double* g, double* w,
                    hipStream_t st) {
  void* base = nullptr;
  TRY_ST(scratch_ptr(&base));
  int ni[3] = {1, 1, 1}, N[3] = {2, 2, 2};
  double h[3] = {1, 1, 1};
  for (int a = 0; a < dim; ++a) {
    N[a] = n[a];
    ni[a] = n[a] - 1;
    h[a] = (hi[a] - lo[a]) / n[a];
  }
  const long long px = ((ni[0] + 31) / 32) * 32;
  const long long nalloc = px * ni[1] * ni[2];
  if (NOALLOC_TABLE_BYTES + (size_t)nalloc * sizeof(T) > NOALLOC_SCRATCH_BYTES) {
    set_last_error("grid too large for the no-alloc scratch array (64 MiB: work array of the padded interior "
                   "plus 1 MiB of tables)",
                   "ahoc_poisson_noalloc");
    return ST_INVALID;
  }
  unsigned char* p = static_cast<unsigned char*>(base);
  size_t off = 0;
  DstTables<T> tb[3];
  T* s[3] = {nullptr, nullptr, nullptr};
  for (int a = 0; a < dim; ++a) {
    const int ppt = dst_ppt(N[a]);
    tb[a].N = N[a];
    tb[a].ppt = ppt;
    if (ppt) {
      // the radix plan of the FFT kernels (host data only)
      DstTables<T> tmp;
      TRY_ST(dst_plan_only<T>(tmp, N[a]));
      tb[a].nrad = tmp.nrad;
      for (int r = 0; r < tmp.nrad; ++r) tb[a].rad[r] = tmp.rad[r];
      tb[a].tw = reinterpret_cast<cx<T>*>(p + off);
      off = align256(off + sizeof(cx<T>) * N[a]);
    }
    tb[a].sn = reinterpret_cast<T*>(p + off);
    off = align256(off + sizeof(T) * (ppt ? N[a] / 2 + 1 : 2 * (size_t)N[a]));
    s[a] = reinterpret_cast<T*>(p + off);
    off = align256(off + sizeof(T) * ni[a]);
    if (off > NOALLOC_TABLE_BYTES) return ST_INVALID;  // cannot happen for N <= 8192
    const int total = (ppt ? N[a] : 0) + (ppt ? N[a] / 2 + 1 : 2 * N[a]) + ni[a];
    hipLaunchKernelGGL((k_axis_tables<T>), dim3((total + 255) / 256), dim3(256), 0, st, N[a], ppt ? 1 : 0, h[a],
                       tb[a].tw, tb[a].sn, s[a]);
    AHOC_HIP_TRY(hipGetLastError());
  }
  T* buf = reinterpret_cast<T*>(p + NOALLOC_TABLE_BYTES);
  // eigen scaling of the slowest-axis pass: lambda = A + B s_t with the other axes' s
  double norm = 1.0;
  for (int a = 0; a < dim; ++a) norm *= 2.0 / N[a];
  const int t = dim - 1;
  DstScale<T> sc;
  sc.s_this = s[t];
  sc.s_a = s[0];
  sc.na = (int)px;
  sc.nva = ni[0];
  if (dim == 3) {
    sc.s_b = s[1];
    sc.c_ta = (T)((h[2] * h[2] + h[0] * h[0]) / 12.0);
    sc.c_tb = (T)((h[2] * h[2] + h[1] * h[1]) / 12.0);
    sc.c_ab = (T)((h[0] * h[0] + h[1] * h[1]) / 12.0);
  } else {
    sc.s_b = nullptr;
    sc.c_ta = (T)((h[1] * h[1] + h[0] * h[0]) / 12.0);
  }
  sc.scale = (T)norm;
  const long long rows = (long long)ni[1] * ni[2];
  {
    const long long n = rows * px;
    const unsigned blocks = (unsigned)std::min<long long>((n + 255) / 256, 65536);
    hipLaunchKernelGGL((k_load_padded<T>), dim3(blocks), dim3(256), 0, st, rows, ni[0], (int)px, g, buf);
    AHOC_HIP_TRY(hipGetLastError());
  }
  if (dim == 2) {
    TRY_ST(dst_pass<T>(tb[0], buf, buf, ni[1], 1, px, nullptr, 0, st));
    TRY_ST(dst_pass<T>(tb[1], buf, buf, 1, px, px, &sc, 0, st));
    TRY_ST(dst_pass<T>(tb[0], buf, buf, ni[1], 1, px, nullptr, 0, st));
  } else {
    TRY_ST(dst_pass<T>(tb[0], buf, buf, rows, 1, px, nullptr, 0, st));
    TRY_ST(dst_pass<T>(tb[1], buf, buf, ni[2], px, px, nullptr, 0, st));
    TRY_ST(dst_pass<T>(tb[2], buf, buf, 1, px * ni[1], px, &sc, 0, st));
    TRY_ST(dst_pass<T>(tb[1], buf, buf, ni[2], px, px, nullptr, 0, st));
    TRY_ST(dst_pass<T>(tb[0], buf, buf, rows, 1, px, nullptr, 0, st));
  }
  TRY_ST((pitch_copy<T, double>(rows, ni[0], buf, px, w, ni[0], st)));
  // the tables point into the scratch array: nothing to release
  tb[0].tw = tb[1].tw = tb[2].tw = nullptr;
  tb[0].sn = tb[1].sn = tb[2].sn = nullptr;
  return ST_OK;
}

}  // namespace
}  // namespace ahoc

extern "C" ahoc_status ahoc_poisson_noalloc(int precision, int dim, const int* n, const double* lo, const double* hi,
                                            const double* g, double* w, void* stream) {
  if (!n || !lo || !hi || !g || !w || (dim != 2 && dim != 3)) {
    ahoc::set_last_error("bad argument (dim 2 or 3, non-NULL n, lo, hi, g, w)", "ahoc_poisson_noalloc");
    return AHOC_E_INVALID;
  }
  for (int a = 0; a < dim; ++a) {
    if (n[a] < 4 || n[a] > ahoc::DST_MAX_N || !(hi[a] > lo[a])) {
      ahoc::set_last_error("need 4 <= n[a] <= 8192 and hi > lo", "ahoc_poisson_noalloc");
      return AHOC_E_INVALID;
    }
  }
  const hipStream_t st = (hipStream_t)stream;
  int rc;
  if (precision == AHOC_FP64) rc = ahoc::poisson_noalloc<double>(dim, n, lo, hi, g, w, st);
  else if (precision == AHOC_MIXED) rc = ahoc::poisson_noalloc<float>(dim, n, lo, hi, g, w, st);
  else {
    ahoc::set_last_error("precision must be AHOC_FP64 or AHOC_MIXED", "ahoc_poisson_noalloc");
    return AHOC_E_INVALID;
  }
  return (ahoc_status)rc;
}
