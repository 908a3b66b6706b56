// Copy kernels that calibrate the bandwidth the DST passes can reach on the device: a plain
// linear copy, and copies with the global access pattern of the strided passes (tiles of
// 16 column pairs = 128 B segments of FP32 rows, 1024 threads, persistent), along the middle
// axis (rows of one plane) and along the slowest axis (across planes).  No arithmetic: the
// time is what HBM takes for the same bytes in the same pattern.  Arrays of at least
// NT_STORE_MIN_BYTES are copied with non-temporal loads and stores, the policy of the passes
// at that size, and every thread has several loads in flight before its stores (one box,
// 8.6 GB moved: linear 5.70 TB/s, 5.50 with the default policy, 4.90 with one 16-byte
// vector per thread at a time; tiles 4.44, 4.42 with the default policy).
#include "common.h"
#include "dst_device.h"

namespace ahoc {

namespace {

constexpr int CT = 1024;   // threads per work-group of the tile copies
constexpr int CQ = 16;     // column pairs per tile
constexpr int CU = 16;     // rows per thread per round
typedef float F2 __attribute__((ext_vector_type(2)));

// tile = (slab o, column tile): columns c0 .. c0+2 CQ-1 of the `rows` rows, `stride` floats
// apart, of slab o (slabs `slab` floats apart)
template <bool NT>
__global__ void __launch_bounds__(CT) k_copy_tiles(const float* __restrict__ in, float* __restrict__ out,
                                                   long long ntiles, long long tiles_per_slab, long long slab,
                                                   long long stride, int rows) {
  const int q = threadIdx.x % CQ, mi = threadIdx.x / CQ;
  constexpr int RSTEP = CT / CQ;
  for (long long t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const long long o = t / tiles_per_slab;
    const long long c0 = (t - o * tiles_per_slab) * (2 * CQ);
    const float2* src = reinterpret_cast<const float2*>(in + o * slab + c0) + q;
    float2* dst = reinterpret_cast<float2*>(out + o * slab + c0) + q;
    const long long st2 = stride / 2;
    // lanes past the last row copy the last row again (the same value to the same place):
    // no predicated accesses, so all loads of a round are in flight before the stores
    for (int rb = 0; rb < rows; rb += CU * RSTEP) {
      float2 v[CU];
#pragma unroll
      for (int u = 0; u < CU; ++u) {
        const float2* p = src + min(rb + mi + u * RSTEP, rows - 1) * st2;
        if constexpr (NT) v[u] = __builtin_bit_cast(float2, __builtin_nontemporal_load(reinterpret_cast<const F2*>(p)));
        else v[u] = *p;
      }
#pragma unroll
      for (int u = 0; u < CU; ++u) {
        float2* p = dst + min(rb + mi + u * RSTEP, rows - 1) * st2;
        if constexpr (NT) __builtin_nontemporal_store(__builtin_bit_cast(F2, v[u]), reinterpret_cast<F2*>(p));
        else *p = v[u];
      }
    }
  }
}

// linear: rounds of LU x 256 16-byte vectors per work-group, the round's loads issued before its stores
constexpr int LU = 4;
template <bool NT>
__global__ void __launch_bounds__(256) k_copy_linear(const float* __restrict__ in, float* __restrict__ out,
                                                     long long n4) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const f4* src = reinterpret_cast<const f4*>(in);
  f4* dst = reinterpret_cast<f4*>(out);
  for (long long base = blockIdx.x * (256LL * LU); base < n4; base += (long long)gridDim.x * (256 * LU)) {
    f4 v[LU];
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      const long long i = base + u * 256 + threadIdx.x;
      if (i < n4) {
        if constexpr (NT) v[u] = __builtin_nontemporal_load(src + i);
        else v[u] = src[i];
      }
    }
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      const long long i = base + u * 256 + threadIdx.x;
      if (i < n4) {
        if constexpr (NT) __builtin_nontemporal_store(v[u], dst + i);
        else dst[i] = v[u];
      }
    }
  }
}

}  // namespace

int copy_bandwidth(int pattern, const float* in, float* out, int nx, int ny, int nz, hipStream_t st) {
  if (!in || !out || nx <= 0 || ny <= 0 || nz <= 0 || nx % (2 * CQ) != 0) return ST_INVALID;
  const long long plane = (long long)nx * ny;
  const bool nt = (double)plane * nz * sizeof(float) >= fast::NT_STORE_MIN_BYTES;
  if (pattern == 0) {
    const long long n = plane * nz;
    if (n % 4) return ST_INVALID;
    const long long n4 = n / 4;
    const long long blocks = std::max(1LL, std::min(32768LL, (n4 + 256 * LU - 1) / (256 * LU)));
    if (nt)
      hipLaunchKernelGGL(k_copy_linear<true>, dim3((unsigned)blocks), dim3(256), 0, st, in, out, n4);
    else
      hipLaunchKernelGGL(k_copy_linear<false>, dim3((unsigned)blocks), dim3(256), 0, st, in, out, n4);
  } else if (pattern == 1) {  // along y: rows of a plane, tiles of columns per plane
    const long long tps = nx / (2 * CQ);
    if (nt)
      hipLaunchKernelGGL(k_copy_tiles<true>, dim3(512), dim3(CT), 0, st, in, out, (long long)nz * tps, tps, plane,
                         (long long)nx, ny);
    else
      hipLaunchKernelGGL(k_copy_tiles<false>, dim3(512), dim3(CT), 0, st, in, out, (long long)nz * tps, tps, plane,
                         (long long)nx, ny);
  } else if (pattern == 2) {  // along z: one slab, tiles of the (y, x) plane's columns
    const long long tps = plane / (2 * CQ);
    if (nt)
      hipLaunchKernelGGL(k_copy_tiles<true>, dim3(512), dim3(CT), 0, st, in, out, tps, tps, 0LL, plane, nz);
    else
      hipLaunchKernelGGL(k_copy_tiles<false>, dim3(512), dim3(CT), 0, st, in, out, tps, tps, 0LL, plane, nz);
  } else {
    return ST_INVALID;
  }
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

}  // namespace ahoc
