// DST-I of short pencils as dense products on the matrix cores (gfx950 MFMA).
//
// For even N <= 128 the transform X_k = sum_{m=1}^{N-1} x_m sin(pi k m / N) (the sine
// diagonalisation of Sec. 2.3) is applied as two half-size products.  With H = N/2 and
// sin(pi k (N-m) / N) = (-1)^(k+1) sin(pi k m / N):
//   odd k = 2j+1:   X_k = sum_{m=1}^{H}   e_m sin(pi (2j+1) m / N),  e_m = x_m + x_{N-m} (m < H), e_H = x_H
//   even k = 2j:    X_k = sum_{m=1}^{H-1} o_m sin(pi 2j m / N),      o_m = x_m - x_{N-m}
// i.e. about N^2 flops per pencil instead of 2 N^2 for the full sine matrix (against the
// FFT's ~2.5 N log2(2N)), on the matrix cores, with no shuffle or prefix-sum stages.
// A work-group has one wavefront per 16 outputs of either half; each wavefront keeps its
// 16 columns of the half matrix in registers as one MFMA operand for the work-group's
// (persistent) lifetime, and streams tiles of pencils through LDS as the other, the
// combinations e, o formed while loading.  Accumulation is in the working precision
// (v_mfma_f32_16x16x4_f32, v_mfma_f64_16x16x4_f64).  Whether a pass uses it is decided at
// setup by timing it against the FFT kernels on the actual shape (dst_tune.hip).
#include "common.h"

#include <cmath>
#include <vector>

namespace ahoc {

namespace {

template <typename T> struct Mfma;
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of the 16x16 result held in element r of lane group lk = lane / 16
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
  static constexpr int XPAD = 4;  // rows-kind LDS row padding (words) -> conflict-free A reads
};
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
  static constexpr int XPAD = 2;
};

constexpr int MAX_GRID = 2048;
// strided-kind LDS row length for TP columns: 16 (mod 64) words apart -> conflict-free B reads
template <int TP> constexpr int cols_ldc() { return TP == 16 ? 16 : TP + 16; }

// 16x16x4 operand layout: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]; element r
// of its result 4-vector is D[i][l % 16] with i = 4 (l / 16) + r for the FP32 instruction
// and i = l / 16 + 4 r for the FP64 one (Mfma<T>::row).
//
// Half matrices (device table, [2][HP][HP], zero-padded): part 0 M0[m-1][j] =
// sin(pi (2j+1) m / N) (m, j+1 <= H), part 1 M1[m-1][j-1] = sin(pi 2j m / N) (m, j <= H-1).
// Wavefront w < HP/16 computes odd outputs 2j+1, j in [16w, 16w+16); wavefront HP/16 + b
// computes even outputs 2j, j - 1 in [16b, 16b+16).  Output k is stored at position k-1.

// Contiguous pencils: rows r0 .. r0+TP-1 of a tile.  in may equal out: a tile's rows are
// read into LDS before any of them is written, and tiles are disjoint.
template <typename T, int HP, int TP>
__global__ void __launch_bounds__(HP / 8 * 64) k_dst_gemm_rows(const T* __restrict__ in, T* __restrict__ out,
                                                               const T* __restrict__ S, long long nrows,
                                                               long long pitch, int N, long long ntiles) {
  using M = Mfma<T>;
  constexpr int NT = HP / 8 * 64;
  constexpr int LDX = HP + M::XPAD;
  constexpr int YS = 2 * LDX;  // output staging row (reuses both halves' tiles)
  __shared__ T zs[2 * TP * LDX];
  const int H = N / 2, L = N - 1;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int part = w < HP / 16 ? 0 : 1;
  const int jb = part ? w - HP / 16 : w;
  T sb[HP / 4];  // B operands: M_part[4 s + lk][16 jb + li]
#pragma unroll
  for (int s = 0; s < HP / 4; ++s) sb[s] = S[part * HP * HP + (4 * s + lk) * HP + 16 * jb + li];
  const int j = 16 * jb + li;
  const int col = part ? 2 * j + 1 : 2 * j;           // output position k-1
  const bool colok = part ? j < H - 1 : j < H;
  const T* zp = zs + part * TP * LDX;
  for (long long t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const long long r0 = t * TP;
    for (int e = threadIdx.x; e < TP * HP; e += NT) {
      const int r = e / HP, q = e - r * HP;  // q = m - 1
      T a = T(0), b = T(0);
      if (q < H && r0 + r < nrows) {
        const T* rp = in + (r0 + r) * pitch;
        a = rp[q];
        if (q < H - 1) b = rp[N - q - 2];
      }
      zs[r * LDX + q] = a + b;
      zs[TP * LDX + r * LDX + q] = a - b;
    }
    __syncthreads();
    typename M::v4 acc[TP / 16];
#pragma unroll
    for (int b = 0; b < TP / 16; ++b) acc[b] = typename M::v4{T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int s = 0; s < HP / 4; ++s) {
#pragma unroll
      for (int b = 0; b < TP / 16; ++b) acc[b] = M::op(zp[(16 * b + li) * LDX + 4 * s + lk], sb[s], acc[b]);
    }
    __syncthreads();  // staging overwrites the tiles
    if (colok) {
#pragma unroll
      for (int b = 0; b < TP / 16; ++b) {
#pragma unroll
        for (int r = 0; r < 4; ++r) zs[(16 * b + M::row(lk, r)) * YS + col] = acc[b][r];
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < TP * 2 * HP; e += NT) {
      const int r = e / (2 * HP), c = e - r * (2 * HP);
      if (c < L && r0 + r < nrows) out[(r0 + r) * pitch + c] = zs[r * YS + c];
    }
    __syncthreads();  // the next tile overwrites the staging rows
  }
}

// Strided pencils, layout [outer][N-1][inner]: the TP columns j of a tile.  in may equal
// out (as above).
template <typename T, int HP, int TP>
__global__ void __launch_bounds__(HP / 8 * 64) k_dst_gemm_cols(const T* __restrict__ in, T* __restrict__ out,
                                                               const T* __restrict__ S, long long inner, int N,
                                                               long long ntile_inner, long long ntiles) {
  using M = Mfma<T>;
  constexpr int NT = HP / 8 * 64;
  constexpr int LDC = cols_ldc<TP>();
  __shared__ T zs[2 * HP * LDC];
  const int H = N / 2, L = N - 1;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int part = w < HP / 16 ? 0 : 1;
  const int jb = part ? w - HP / 16 : w;
  T sa[HP / 4];  // A operands: M_part[4 s + lk][16 jb + li] (transposed read)
#pragma unroll
  for (int s = 0; s < HP / 4; ++s) sa[s] = S[part * HP * HP + (4 * s + lk) * HP + 16 * jb + li];
  const T* zp = zs + part * HP * LDC;
  for (long long t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const long long o = t / ntile_inner;
    const long long c0 = (t - o * ntile_inner) * TP;
    const long long base = o * (long long)L * inner;  // slab o
    for (int e = threadIdx.x; e < HP * TP; e += NT) {
      const int q = e / TP, c = e - q * TP;
      T a = T(0), b = T(0);
      if (q < H && c0 + c < inner) {
        a = in[base + (long long)q * inner + c0 + c];
        if (q < H - 1) b = in[base + (long long)(N - q - 2) * inner + c0 + c];
      }
      zs[q * LDC + c] = a + b;
      zs[HP * LDC + q * LDC + c] = a - b;
    }
    __syncthreads();
    typename M::v4 acc[TP / 16];
#pragma unroll
    for (int b = 0; b < TP / 16; ++b) acc[b] = typename M::v4{T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int s = 0; s < HP / 4; ++s) {
#pragma unroll
      for (int b = 0; b < TP / 16; ++b) acc[b] = M::op(sa[s], zp[(4 * s + lk) * LDC + 16 * b + li], acc[b]);
    }
    __syncthreads();  // the next tile overwrites zs
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int jj = 16 * jb + M::row(lk, r);
      const int k1 = part ? 2 * jj + 1 : 2 * jj;  // output position k-1
      if (part ? jj < H - 1 : jj < H) {
#pragma unroll
        for (int b = 0; b < TP / 16; ++b) {
          const long long c = c0 + 16 * b + li;
          if (c < inner) out[base + (long long)k1 * inner + c] = acc[b][r];
        }
      }
    }
  }
}

template <typename T, int HP, int TP>
void gemm_launch_tp(const T* S, int N, const T* in, T* out, long long outer, long long inner, long long pitch,
                    hipStream_t st) {
  constexpr int NT = HP / 8 * 64;
  if (inner == 1) {
    const long long ntiles = (outer + TP - 1) / TP;
    const unsigned grid = (unsigned)std::min<long long>(ntiles, MAX_GRID);
    hipLaunchKernelGGL((k_dst_gemm_rows<T, HP, TP>), dim3(grid), dim3(NT), 0, st, in, out, S, outer, pitch, N,
                       ntiles);
  } else {
    const long long nti = (inner + TP - 1) / TP;
    const long long ntiles = outer * nti;
    const unsigned grid = (unsigned)std::min<long long>(ntiles, MAX_GRID);
    hipLaunchKernelGGL((k_dst_gemm_cols<T, HP, TP>), dim3(grid), dim3(NT), 0, st, in, out, S, inner, N, nti,
                       ntiles);
  }
}

// Tiles of 64 pencils; 16-pencil tiles (four times the work-groups, a quarter of the MFMA
// chain per wavefront) when a pass has fewer 64-pencil tiles than two per compute unit.
template <typename T, int HP>
int gemm_launch(const T* S, int N, const T* in, T* out, long long outer, long long inner, long long pitch,
                hipStream_t st) {
  const long long n64 = inner == 1 ? (outer + 63) / 64 : outer * ((inner + 63) / 64);
  if (n64 <= 0) return ST_OK;
  if (n64 < 512) gemm_launch_tp<T, HP, 16>(S, N, in, out, outer, inner, pitch, st);
  else gemm_launch_tp<T, HP, 64>(S, N, in, out, outer, inner, pitch, st);
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

}  // namespace

bool dst_gemm_supported(int N) { return N >= 4 && N <= DST_GEMM_MAX_N && N % 2 == 0; }

// padded half length HP = 16 ceil(N / 32)
int dst_gemm_hp(int N) { return dst_gemm_supported(N) ? (N / 2 + 15) / 16 * 16 : 0; }

template <typename T> int dst_gemm_table(T** S, int N, hipStream_t st, const DevAlloc& al) {
  *S = nullptr;
  const int HP = dst_gemm_hp(N);
  if (!HP) return ST_UNSUPPORTED;
  const int H = N / 2;
  std::vector<T> h(2 * (size_t)HP * HP, T(0));
  const long double pi = 3.141592653589793238462643383279502884L;
  // sin(pi p / N) has period 2N in p: reduce the integer argument first
  auto sn = [&](long long p) { return (T)sinl(pi * (long double)(p % (2LL * N)) / (long double)N); };
  for (int m = 1; m <= H; ++m)
    for (int j = 0; j < H; ++j) h[(size_t)(m - 1) * HP + j] = sn((long long)(2 * j + 1) * m);
  for (int m = 1; m <= H - 1; ++m)
    for (int j = 1; j <= H - 1; ++j) h[(size_t)HP * HP + (size_t)(m - 1) * HP + (j - 1)] = sn(2LL * j * m);
  {
    const int rc = dev_alloc(al, reinterpret_cast<void**>(S), sizeof(T) * h.size());
    if (rc != ST_OK) return rc;
  }
  AHOC_HIP_TRY(hipMemcpyAsync(*S, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, st));
  AHOC_HIP_TRY(hipStreamSynchronize(st));
  return ST_OK;
}

template <typename T>
int dst_gemm_pass(const T* S, int N, const T* in, T* out, long long outer, long long inner, long long pitch,
                  hipStream_t st) {
  if (!S || !dst_gemm_supported(N)) return ST_UNSUPPORTED;
  if (outer < 0 || inner < 1 || (inner == 1 && pitch < N - 1)) return ST_INVALID;
  switch (dst_gemm_hp(N)) {
    case 16: return gemm_launch<T, 16>(S, N, in, out, outer, inner, pitch, st);
    case 32: return gemm_launch<T, 32>(S, N, in, out, outer, inner, pitch, st);
    case 48: return gemm_launch<T, 48>(S, N, in, out, outer, inner, pitch, st);
    case 64: return gemm_launch<T, 64>(S, N, in, out, outer, inner, pitch, st);
    default: return ST_UNSUPPORTED;
  }
}

template int dst_gemm_table<float>(float**, int, hipStream_t, const DevAlloc&);
template int dst_gemm_table<double>(double**, int, hipStream_t, const DevAlloc&);
template int dst_gemm_pass<float>(const float*, int, const float*, float*, long long, long long, long long,
                                  hipStream_t);
template int dst_gemm_pass<double>(const double*, int, const double*, double*, long long, long long, long long,
                                   hipStream_t);

}  // namespace ahoc
