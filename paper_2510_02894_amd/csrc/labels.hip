// labels.hip -- input preprocessing on the device: the bounding box and voxel
// count of every label of a uint8 label map in one read of the map, written
// as a device ROI table (crop to the box, select the label) that the batched
// pipeline consumes directly.  The paper leaves reading and staging the
// input on the host as its open problem (Sec. 3, discussion of the results,
// and the transfer column of Table 2); this keeps that step on the GPU.
#include <climits>

#include "s3d_launch.h"

namespace s3d {

namespace {

constexpr int kLabelThreads = 256;

// The box under construction for one label: per-thread registers first, then
// the workgroup's LDS entry, then the global one.
struct RegBox {
  int l;  // 0 = empty
  int lo[3], hi[3];
  unsigned long long n;
};

__device__ inline void flush_box(RegBox& b, int* s_lo, int* s_hi, unsigned long long* s_n) {
  if (b.l) {
    const int i = b.l - 1;
    for (int k = 0; k < 3; ++k) {
      atomicMin(&s_lo[3 * i + k], b.lo[k]);
      atomicMax(&s_hi[3 * i + k], b.hi[k]);
    }
    atomicAdd(&s_n[i], b.n);
  }
  b.l = 0;
}

__device__ inline void add_run(RegBox& b, int l, int z, int y, int x0, int x1, unsigned long long n, int* s_lo,
                               int* s_hi, unsigned long long* s_n) {
  if (l != b.l) {
    flush_box(b, s_lo, s_hi, s_n);
    b.l = l;
    b.lo[0] = z;
    b.lo[1] = y;
    b.lo[2] = x0;
    b.hi[0] = z;
    b.hi[1] = y;
    b.hi[2] = x1;
    b.n = n;
    return;
  }
  b.lo[0] = min(b.lo[0], z);
  b.lo[1] = min(b.lo[1], y);
  b.lo[2] = min(b.lo[2], x0);
  b.hi[0] = max(b.hi[0], z);
  b.hi[1] = max(b.hi[1], y);
  b.hi[2] = max(b.hi[2], x1);
  b.n += n;
}

// Row-major coordinates of voxel j (0 <= j < d0 d1 d2): floating-point
// quotients, corrected by one step either way (j < 2^53).
__device__ inline void voxel_coords(long long j, long long d12, int d1, int d2, double inv12, double inv2, int& z,
                                    int& y, int& x) {
  long long q = (long long)((double)j * inv12);
  if (q * d12 > j) --q;
  if ((q + 1) * d12 <= j) ++q;
  const long long r = j - q * d12;
  long long p = (long long)((double)r * inv2);
  if (p * d2 > r) --p;
  if ((p + 1) * d2 <= r) ++p;
  z = (int)q;
  y = (int)p;
  x = (int)(r - p * d2);
}

// The boxes under construction live in the first 32 bytes of the output
// table's entries (an 80-byte RoiDesc per label), so the pass needs no
// memory of its own; the table kernel replaces each by the finished entry.
__device__ inline LabelAcc* acc_of(RoiDesc* tab, int i) { return reinterpret_cast<LabelAcc*>(tab + i); }

}  // namespace

// Clears the boxes of labels 1..max_label.
__global__ void k_label_init(RoiDesc* __restrict__ tab, int max_label) {
  const int i = threadIdx.x;
  if (i < max_label) {
    LabelAcc* a = acc_of(tab, i);
    for (int k = 0; k < 3; ++k) {
      a->lo[k] = INT_MAX;
      a->hi[k] = -1;
    }
    a->n = 0ull;
  }
}

// One read of the map in 16-byte chunks, addressed from the 16-byte aligned
// address at or below lab.  Chunks wholly inside the map are one vector load;
// the two partial chunks at the ends are read byte by byte.  A chunk of 16
// equal labels inside one row is one run; other chunks are walked voxel by
// voxel.  Each thread keeps the box of its current label in registers and
// folds it into the workgroup's LDS boxes when the label changes; the
// workgroup's boxes go to memory with one set of atomics per label present.
__global__ __launch_bounds__(kLabelThreads) void k_label_boxes(const unsigned char* __restrict__ lab, long long n,
                                                               int mis, long long d12, int d1, int d2, double inv12,
                                                               double inv2, int max_label,
                                                               RoiDesc* __restrict__ tab) {
  __shared__ int s_lo[255 * 3], s_hi[255 * 3];
  __shared__ unsigned long long s_n[255];
  for (int i = threadIdx.x; i < max_label; i += blockDim.x) {
    for (int k = 0; k < 3; ++k) {
      s_lo[3 * i + k] = INT_MAX;
      s_hi[3 * i + k] = -1;
    }
    s_n[i] = 0ull;
  }
  __syncthreads();
  RegBox b;
  b.l = 0;
  const unsigned char* p0 = lab - mis;
  const long long nchunks = (n + mis + 15) >> 4;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < nchunks; c += stride) {
    const long long j0 = c * 16 - mis;  // voxel index of the chunk's first byte
    unsigned int w[4];
    int k0 = 0, k1 = 16;
    if (j0 >= 0 && j0 + 16 <= n) {
      const uint4 v = *(const uint4*)(p0 + c * 16);
      w[0] = v.x;
      w[1] = v.y;
      w[2] = v.z;
      w[3] = v.w;
    } else {
      k0 = j0 < 0 ? (int)(-j0) : 0;
      k1 = (int)min(16ll, n - j0);
      for (int q = 0; q < 4; ++q) w[q] = 0u;
      for (int k = k0; k < k1; ++k) w[k >> 2] |= (unsigned int)p0[c * 16 + k] << (8 * (k & 3));
    }
    if ((w[0] | w[1] | w[2] | w[3]) == 0u) continue;
    int z, y, x;
    voxel_coords(j0 + k0, d12, d1, d2, inv12, inv2, z, y, x);
    const unsigned int l0 = w[0] & 0xFFu;
    if (k0 == 0 && k1 == 16 && l0 != 0u && (int)l0 <= max_label && x + 15 < d2 && w[0] == l0 * 0x01010101u &&
        w[1] == w[0] && w[2] == w[0] && w[3] == w[0]) {
      add_run(b, (int)l0, z, y, x, x + 15, 16ull, s_lo, s_hi, s_n);
      continue;
    }
    for (int k = k0; k < k1; ++k) {
      const int l = (int)((w[k >> 2] >> (8 * (k & 3))) & 0xFFu);
      if (l != 0 && l <= max_label) add_run(b, l, z, y, x, x, 1ull, s_lo, s_hi, s_n);
      if (++x == d2) {
        x = 0;
        if (++y == d1) {
          y = 0;
          ++z;
        }
      }
    }
  }
  flush_box(b, s_lo, s_hi, s_n);
  __syncthreads();
  for (int i = threadIdx.x; i < max_label; i += blockDim.x) {
    if (s_n[i] == 0ull) continue;
    LabelAcc* a = acc_of(tab, i);
    for (int k = 0; k < 3; ++k) {
      atomicMin(&a->lo[k], s_lo[3 * i + k]);
      atomicMax(&a->hi[k], s_hi[3 * i + k]);
    }
    atomicAdd(&a->n, s_n[i]);
  }
}

// The ROI table (one workgroup): label l's entry crops the map to the label's
// box; a label with no voxel gets a 1-voxel crop at the origin (which then
// holds no voxel of it).  max_dims: the largest crop along each axis.
__global__ void k_label_table(RoiDesc* __restrict__ rois, int max_label, long long d1, long long d2, double s0,
                              double s1, double s2, long long* __restrict__ counts,
                              long long* __restrict__ max_dims) {
  __shared__ int s_max[3];
  const int i = threadIdx.x;
  if (i < 3) s_max[i] = 1;
  __syncthreads();
  if (i < max_label) {
    const LabelAcc a = *acc_of(rois, i);  // read before the entry is overwritten
    RoiDesc R;
    R.spacing[0] = s0;
    R.spacing[1] = s1;
    R.spacing[2] = s2;
    R.strides[0] = d1 * d2;
    R.strides[1] = d2;
    R.label = i + 1;
    R.reserved = 0;
    if (a.n == 0ull) {
      R.offset = 0;
      for (int k = 0; k < 3; ++k) R.dims[k] = 1;
    } else {
      R.offset = (long long)a.lo[0] * d1 * d2 + (long long)a.lo[1] * d2 + a.lo[2];
      for (int k = 0; k < 3; ++k) {
        R.dims[k] = (long long)(a.hi[k] - a.lo[k] + 1);
        atomicMax(&s_max[k], a.hi[k] - a.lo[k] + 1);
      }
    }
    rois[i] = R;
    if (counts) counts[i] = (long long)a.n;
  }
  __syncthreads();
  if (max_dims && i < 3) max_dims[i] = s_max[i];
}

hipError_t launch_label_rois(const unsigned char* lab, const long long dims[3], const double spacing[3],
                             int max_label, RoiDesc* rois, long long* counts, long long* max_dims, int cu_count,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_label_init, dim3(1), dim3(256), 0, st, rois, max_label);
  const long long n = dims[0] * dims[1] * dims[2];
  const int mis = (int)((uintptr_t)lab & 15);
  const long long nchunks = (n + mis + 15) >> 4;
  // about 8 chunks per thread: few LDS-to-global folds, enough waves in flight
  long long grid = (nchunks + 8ll * kLabelThreads - 1) / (8ll * kLabelThreads);
  grid = std::max(1ll, std::min(grid, 16ll * cu_count));
  const long long d12 = dims[1] * dims[2];
  hipLaunchKernelGGL(k_label_boxes, dim3((unsigned)grid), dim3(kLabelThreads), 0, st, lab, n, mis, d12,
                     (int)dims[1], (int)dims[2], 1.0 / (double)d12, 1.0 / (double)dims[2], max_label, rois);
  hipLaunchKernelGGL(k_label_table, dim3(1), dim3(256), 0, st, rois, max_label, dims[1], dims[2], spacing[0],
                     spacing[1], spacing[2], counts, max_dims);
  return hipGetLastError();
}

}  // namespace s3d
