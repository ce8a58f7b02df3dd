// scan.hip -- device-wide exclusive prefix sum of int64 and fill kernels.
#include <hip/hip_runtime.h>

#include "s3d_device.h"
#include "s3d_launch.h"

namespace s3d {

constexpr int kScanThreads = 256;
constexpr int kScanPer = kScanTile / kScanThreads;  // 8 consecutive elements per thread

// The number of elements to scan: n, or fewer when the device holds a smaller
// count (elements past it are treated as absent: their tiles sum to zero and
// their outputs are not written).
__device__ inline long long scan_count(long long n, const unsigned int* n_dev) {
  return n_dev ? min(n, (long long)*n_dev) : n;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const long long* __restrict__ in, long long n,
                                                              const unsigned int* __restrict__ n_dev,
                                                              long long* __restrict__ blk) {
  __shared__ long long sh[4];
  n = scan_count(n, n_dev);
  const long long base = (long long)blockIdx.x * kScanTile;
  if (base >= n && blockIdx.x > 0) {
    if (threadIdx.x == 0) blk[blockIdx.x] = 0;
    return;
  }
  long long s = 0;
  for (int i = 0; i < kScanPer; ++i) {
    const long long idx = base + (long long)i * kScanThreads + threadIdx.x;
    if (idx < n) s += in[idx];
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) blk[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// In-place exclusive scan of nb block sums in one workgroup; total -> *total.
__global__ __launch_bounds__(1024) void k_scan_top(long long* __restrict__ blk, long long nb,
                                                   long long* __restrict__ total) {
  __shared__ long long s[2][1024];
  const int tid = threadIdx.x;
  const long long chunk = (nb + 1023) / 1024;
  const long long lo = min(nb, chunk * tid), hi = min(nb, chunk * (tid + 1));
  long long sum = 0;
  for (long long i = lo; i < hi; ++i) sum += blk[i];
  s[0][tid] = sum;
  __syncthreads();
  int src = 0;
  for (int d = 1; d < 1024; d <<= 1) {
    long long v = s[src][tid];
    if (tid >= d) v += s[src][tid - d];
    s[1 - src][tid] = v;
    __syncthreads();
    src = 1 - src;
  }
  long long off = s[src][tid] - sum;
  for (long long i = lo; i < hi; ++i) {
    const long long v = blk[i];
    blk[i] = off;
    off += v;
  }
  if (tid == 1023 && total) *total = s[src][1023];
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const long long* __restrict__ in, long long n,
                                                             const unsigned int* __restrict__ n_dev,
                                                             const long long* __restrict__ blk,
                                                             long long* __restrict__ out) {
  __shared__ long long sh[4];
  n = scan_count(n, n_dev);
  if ((long long)blockIdx.x * kScanTile >= n) return;  // uniform per workgroup
  const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanPer;
  long long v[kScanPer];
  long long s = 0;
  for (int i = 0; i < kScanPer; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0;
    s += v[i];
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  long long inc = s;
  for (int d = 1; d < 64; d <<= 1) {
    long long t = __shfl_up(inc, d, 64);
    if (lane >= d) inc += t;
  }
  if (lane == 63) sh[wid] = inc;
  __syncthreads();
  long long off = blk[blockIdx.x];
  for (int w = 0; w < wid; ++w) off += sh[w];
  off += inc - s;
  for (int i = 0; i < kScanPer; ++i) {
    if (base + i < n) out[base + i] = off;
    off += v[i];
  }
}

// The whole scan in one 1024-thread workgroup, for n <= kScanSingleMax: each
// thread sums a contiguous run of at most 64 elements, the run sums are
// scanned (wave scans, then the 16 wave totals), and each thread writes its
// run.  One launch instead of three for the many small scans of a call.
constexpr long long kScanSingleMax = 1024 * 64;

__global__ __launch_bounds__(1024) void k_scan_single(const long long* __restrict__ in, long long n,
                                                      const unsigned int* __restrict__ n_dev,
                                                      long long* __restrict__ out, long long* __restrict__ total) {
  __shared__ long long sw[16];
  n = scan_count(n, n_dev);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const long long per = (n + 1023) / 1024;
  const long long lo = min(n, per * tid), hi = min(n, lo + per);
  long long sum = 0;
  for (long long i = lo; i < hi; ++i) sum += in[i];
  long long inc = sum;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const long long t = __shfl_up(inc, d, 64);
    if (lane >= d) inc += t;
  }
  if (lane == 63) sw[wid] = inc;
  __syncthreads();
  long long base = 0, all = 0;
  for (int w = 0; w < 16; ++w) {
    if (w < wid) base += sw[w];
    all += sw[w];
  }
  long long off = base + inc - sum;
  for (long long i = lo; i < hi; ++i) {
    const long long v = in[i];
    out[i] = off;
    off += v;
  }
  if (tid == 0 && total) *total = all;
}

long long scan_tmp_elems(long long n) { return (n + kScanTile - 1) / kScanTile + 1; }

hipError_t launch_scan(const long long* in, long long* out, long long n, long long* total, long long* tmp,
                       hipStream_t st, const unsigned int* n_dev) {
  if (n <= kScanSingleMax) {
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, st, in, n, n_dev, out, total);
    return hipGetLastError();
  }
  const long long nb = n > 0 ? (n + kScanTile - 1) / kScanTile : 1;
  if (n > 0) hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, n, n_dev, tmp);
  else hipLaunchKernelGGL(k_scan_reduce, dim3(1), dim3(kScanThreads), 0, st, in, 0ll, n_dev, tmp);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, tmp, nb, total);
  if (n > 0) hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, n, n_dev, tmp, out);
  return hipGetLastError();
}

__global__ void k_fill_u32(unsigned int* p, unsigned int v, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_i64(long long* p, long long v, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

static unsigned fill_grid(long long n) {
  long long g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  return (unsigned)g;
}

hipError_t launch_fill_u32(unsigned int* p, unsigned int v, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid(n)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_i64(long long* p, long long v, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i64, dim3(fill_grid(n)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

}  // namespace s3d
