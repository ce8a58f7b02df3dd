// s3d_device.h -- device helpers shared by the HIP translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "s3d_internal.h"

namespace s3d {

// Maps a workgroup index to a work index so that each of the 8 XCDs (which
// receive workgroups round-robin) walks one contiguous range of work indices:
// neighbouring bricks then share that XCD's L2.  A bijection on [0, n).
__device__ inline long long xcd_remap(long long bid, long long n) {
  const long long per = n / 8, rem = n % 8;
  const long long x = bid % 8, idx = bid / 8;
  return x * per + (x < rem ? x : rem) + idx;
}

// floor(n / d) for 0 <= n < 2^31 from the precomputed pair m = floor(2^sh / d) + 1,
// sh = 31 + ceil(log2 d): (n * m) >> sh (the error term n (m - 2^sh / d) / 2^sh
// stays below 1 / d, so the floor is exact).
__device__ inline unsigned int fdiv(unsigned int n, unsigned int m, int sh) {
  return (unsigned int)(((unsigned long long)n * m) >> sh);
}

// Index of the last ROI whose first brick is <= b (ROIs are sorted by brick_begin).
__device__ inline int find_roi(const Roi* rois, int n, long long b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (rois[mid].brick_begin <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ inline int wave_min(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = min(v, __shfl_xor(v, m, 64));
  return v;
}

__device__ inline int wave_max(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = max(v, __shfl_xor(v, m, 64));
  return v;
}

// Exclusive prefix sum over a 256-thread block; `total` receives the block sum.
// `sh` must hold 4 ints of shared memory.  Contains barriers.
__device__ inline int block_excl_scan256(int v, int* sh, int& total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int t = __shfl_up(inc, d, 64);
    if (lane >= d) inc += t;
  }
  if (lane == 63) sh[wid] = inc;
  __syncthreads();
  int base = 0;
  for (int w = 0; w < wid; ++w) base += sh[w];
  total = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return base + inc - v;
}

// 1 / x in FP64 from the hardware reciprocal estimate and two Newton steps
// (each squares the relative error, which ends far below a unit in the last
// place of a double for the estimate's accuracy; the result may differ from the
// correctly rounded quotient in its last bit); x != 0.
__device__ inline double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// Exact FP64 squared distance in a fixed operation order (no contraction).
__device__ inline double dist2_exact(const double* p, const double* q) {
  double dx = __dsub_rn(p[0], q[0]), dy = __dsub_rn(p[1], q[1]), dz = __dsub_rn(p[2], q[2]);
  return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}

// Physical FP64 position of a vertex from its key and interpolation parameter,
// ((double)u_k + [k == a] * t) * s_k, in that operation order.
__device__ inline void key_position(uint64_t key, double t, const double* s, double* x) {
  const int u2 = (int)(key & 0xFFFFF) - 1;
  const int u1 = (int)((key >> 20) & 0xFFFFF) - 1;
  const int u0 = (int)((key >> 40) & 0xFFFFF) - 1;
  const int a = (int)((key >> 60) & 3);
  x[0] = __dmul_rn(__dadd_rn((double)u0, a == 0 ? t : 0.0), s[0]);
  x[1] = __dmul_rn(__dadd_rn((double)u1, a == 1 ? t : 0.0), s[1]);
  x[2] = __dmul_rn(__dadd_rn((double)u2, a == 2 ? t : 0.0), s[2]);
}

// Binary exponent e of the scale 2^e applied to a ROI's centred coordinates
// before the split-f16 pair pass: with R2 a bound on |x|^2, 64 <= 2^e R < 128,
// so scaled coordinates and |x|^2 (< 2^14) are far inside the f16 range.
__host__ __device__ inline int h_scale_exp(double R2) {
  if (!(R2 > 0.0)) return 0;
  int k;
  (void)frexp(R2, &k);                                  // 2^(k-1) <= R2 < 2^k
  const int half = k >= 0 ? (k + 1) / 2 : -((-k) / 2);  // ceil(k / 2)
  const int e = 7 - half;
  return e < -120 ? -120 : (e > 120 ? 120 : e);
}

// Split-f16 B operand of a row (the pair pass's kernel 1): the centred FP32
// position (x, y, z) and w = |p|^2, scaled by 2^e and 2^(2e), each split into
// h = f16(v) and l = f16(v - h).  A row is 32 contiguous bytes: K entries 0-7
// [h, l, h0, h1] (read by lane row % 32 of the MFMA) and then K entries 8-15
// [h2, 1, 1, w_hi, w_lo, 0, 0, 0] (read by lane 32 + row % 32), so lane l of
// a wave reads uint4 2 (l % 32) + l / 32 of the 32-row block: one contiguous
// 1 KB load per block, and one 32-byte record per row to copy.
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

__device__ inline void write_split_row(uint4* __restrict__ posh, long long row, float fx, float fy, float fz,
                                       float fw, int e) {
  const float x[3] = {ldexpf(fx, e), ldexpf(fy, e), ldexpf(fz, e)};
  const float w = ldexpf(fw, 2 * e);
  _Float16 h[3], l[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    h[c] = (_Float16)x[c];
    l[c] = (_Float16)(x[c] - (float)h[c]);
  }
  const _Float16 wh = (_Float16)w, wl = (_Float16)(w - (float)wh);
  const _Float16 one = (_Float16)1.0f, zero = (_Float16)0.0f;
  const v8h b0 = {h[0], h[1], h[2], l[0], l[1], l[2], h[0], h[1]};
  const v8h b1 = {h[2], one, one, wh, wl, zero, zero, zero};
  uint4* r = posh + 2 * row;
  r[0] = *(const uint4*)&b0;
  r[1] = *(const uint4*)&b1;
}

// uint4 index, within a 32-row block of split-f16 operand rows, that lane l
// passes to the MFMA.
__device__ inline int split_lane_index(int lane) { return 2 * (lane & 31) + (lane >> 5); }

// Copies the pair-pass operands of row src to row dst: the split-f16 B
// operand when posh is set, else the FP32 position block entries.
__device__ inline void copy_row_operands(float* __restrict__ pos, uint4* __restrict__ posh, long long src,
                                         long long dst) {
  if (posh) {
    const uint4* s = posh + 2 * src;
    uint4* d = posh + 2 * dst;
    const uint4 a = s[0], b = s[1];
    d[0] = a;
    d[1] = b;
  } else {
    const float* s = pos + (src >> 4) * 64 + (src & 15);
    float* d = pos + (dst >> 4) * 64 + (dst & 15);
    const float a = s[0], b = s[16], c = s[32], w = s[48];
    d[0] = a;
    d[16] = b;
    d[32] = c;
    d[48] = w;
  }
}

// Canonical id 3 * lin_pad(u) + a of a vertex key for a ROI of dims d.
__device__ inline unsigned long long key_canonical_id(uint64_t key, const int* d) {
  const unsigned long long p2 = key & 0xFFFFF, p1 = (key >> 20) & 0xFFFFF, p0 = (key >> 40) & 0xFFFFF;
  const unsigned long long a = (key >> 60) & 3;
  const unsigned long long lin = (p0 * (unsigned long long)(d[1] + 2) + p1) * (unsigned long long)(d[2] + 2) + p2;
  return 3ull * lin + a;
}

}  // namespace s3d
