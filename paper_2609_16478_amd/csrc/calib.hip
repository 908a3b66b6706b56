// Copy kernels that calibrate the bandwidth the DST passes can reach on the device: a plain
// linear copy, and copies with the global access pattern of the strided passes (tiles of
// 16 column pairs = 128 B segments of FP32 rows, 1024 threads, persistent), along the middle
// axis (rows of one plane) and along the slowest axis (across planes).  No arithmetic: the
// time is what HBM takes for the same bytes in the same pattern.
#include "common.h"

namespace ahoc {

namespace {

constexpr int CT = 1024;   // threads per work-group of the tile copies
constexpr int CQ = 16;     // column pairs per tile
constexpr int CU = 16;     // rows per thread per round

// tile = (slab o, column tile): columns c0 .. c0+2 CQ-1 of the `rows` rows, `stride` floats
// apart, of slab o (slabs `slab` floats apart)
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
      for (int u = 0; u < CU; ++u) v[u] = src[min(rb + mi + u * RSTEP, rows - 1) * st2];
#pragma unroll
      for (int u = 0; u < CU; ++u) dst[min(rb + mi + u * RSTEP, rows - 1) * st2] = v[u];
    }
  }
}

__global__ void k_copy_linear(const float4* __restrict__ in, float4* __restrict__ out, long long n4) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n4; i += (long long)gridDim.x * blockDim.x)
    out[i] = in[i];
}

}  // namespace

int copy_bandwidth(int pattern, const float* in, float* out, int nx, int ny, int nz, hipStream_t st) {
  if (!in || !out || nx <= 0 || ny <= 0 || nz <= 0 || nx % (2 * CQ) != 0) return ST_INVALID;
  const long long plane = (long long)nx * ny;
  if (pattern == 0) {
    const long long n = plane * nz;
    if (n % 4) return ST_INVALID;
    hipLaunchKernelGGL(k_copy_linear, dim3(8192), dim3(256), 0, st, reinterpret_cast<const float4*>(in),
                       reinterpret_cast<float4*>(out), n / 4);
  } else if (pattern == 1) {  // along y: rows of a plane, tiles of columns per plane
    const long long tps = nx / (2 * CQ);
    hipLaunchKernelGGL(k_copy_tiles, dim3(512), dim3(CT), 0, st, in, out, (long long)nz * tps, tps, plane,
                       (long long)nx, ny);
  } else if (pattern == 2) {  // along z: one slab, tiles of the (y, x) plane's columns
    const long long tps = plane / (2 * CQ);
    hipLaunchKernelGGL(k_copy_tiles, dim3(512), dim3(CT), 0, st, in, out, tps, tps, 0LL, plane, nz);
  } else {
    return ST_INVALID;
  }
  AHOC_HIP_TRY(hipGetLastError());
  return ST_OK;
}

}  // namespace ahoc
