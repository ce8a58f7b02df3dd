// s3d_internal.h -- data layout shared by the kernels and the host driver.
//
// Work layout (all sizes in elements):
//   * mesh pass: a "brick" is kBrickThreads consecutive row-groups x kTZ cube
//     planes of one ROI; a row-group is 32 consecutive cubes along axis 2 of one
//     cube row (axis 1), handled by one thread as bit masks;
//   * vertices live in "rows": layout 0 holds every ROI's vertices (emission
//     order) padded to a multiple of kSegAlign; the plane layouts follow, one
//     padded bucket per plane that holds at least two vertices;
//   * positions are stored in blocks of 16 rows as 64 floats
//     [x0..x15, y0..y15, z0..z15, w0..w15] (centred coordinates, w = |x|^2),
//     which is the operand layout of the 16x16x4 FP32 MFMA;
//   * a "segment" is a contiguous run of rows whose pairs are examined; a
//     "group" is one feature of one ROI (roi * 4 + {0: 3D, 1..3: plane axis}).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace s3d {

constexpr int kBrickThreads = 256;  // threads (row-groups) per brick
constexpr int kTZ = 8;              // cube planes per brick
constexpr int kBlk = 16;            // rows per position block
constexpr int kSegAlign = 32;       // segment rows padded to a multiple of this
constexpr int kMinJchunk = 64;      // smallest column chunk (row blocks) the pair pass may be tuned to
constexpr int kScanTile = 2048;     // elements per block of the device scan
constexpr int kExactChunk = 4096;   // rows per block of the exact refinement
constexpr int kSmallBlocks = 16;    // plane buckets of up to this many 32-row blocks skip the work list
constexpr int kSmallPerWave = 4;    // bucket segments per wave of the small-bucket kernel
constexpr long long kSmallMinBuckets = 1 << 16;  // calls with fewer plane buckets keep them all in the work list
constexpr int kWorkParts = 8;       // work ranges (one per XCD) of the pair pass, each with its own counter
constexpr int kWorkStride = 32;     // words between two work counters (one 128-byte line each)
// Counter block: word 1 candidates, 2 capacity overflow, 3 pruned work items,
// 4 pruned-list overflow; the work counters of the pair pass from word
// kWorkStride, then those of the pruned 3D pass.
constexpr int kCounterWords = kWorkStride * (1 + 2 * kWorkParts);
constexpr int kListCounters = kWorkStride * (1 + kWorkParts);  // first work counter of the pruned 3D pass
constexpr int kPruneSB = 32;          // 32-row blocks per column of the 3D pruning pass (1024 rows)
constexpr int kPruneMinV = 1024;      // ROIs with fewer vertices run their 3D pairs unpruned (prune = 1)
constexpr int kPruneCallMinV = 16384; // a call prunes (prune = 1) when its largest ROI may have this many vertices

// Key of a vertex: edge (u, u + e_a): bits 0..19 u2+1, 20..39 u1+1, 40..59 u0+1, 60..61 a.
__host__ __device__ inline uint64_t pack_key(int u0, int u1, int u2, int a) {
  return (uint64_t)(uint32_t)(u2 + 1) | ((uint64_t)(uint32_t)(u1 + 1) << 20) |
         ((uint64_t)(uint32_t)(u0 + 1) << 40) | ((uint64_t)a << 60);
}

struct Roi {
  const void* vol;        // this ROI's first voxel (uint8 or float32)
  int d[3];
  int G;                  // row-groups per cube row: ceil((d2 + 1) / 32)
  double s[3];
  long long brick_begin;  // first brick
  long long brick_end;    // one past the last brick
  long long stride0;      // elements between consecutive voxels along axis 0
  long long stride1;      // ... along axis 1 (axis 2 is contiguous)
  int nrg;                // (d1 + 1) * G
  int nzc;                // z-chunks: ceil((d0 + 1) / tz)
  int bpz;                // bricks per z-chunk: ceil(nrg / kBrickThreads)
  int shG;                // floor(n / G) = (n * mG) >> shG for 0 <= n < 2^31
  unsigned int mG;
  unsigned int mNW;       // the same for the tile width kBrickThreads + 1 + G
  int shNW;
  int label;              // uint8 only: 0 = a voxel is inside iff nonzero; else iff it equals label
  int status;             // 0, or a negative status for a rejected table entry (then it has no bricks)
  int tz;                 // cube planes per brick (kTZ, or fewer for a small ROI on its own)
  long long bucket_base[3];  // first global plane bucket of each axis
};

// A ROI as a caller describes it (the layout of shape3d_roi_ex in shape3d.h).
struct RoiDesc {
  long long offset;      // element offset of the ROI's first voxel from the base pointer
  long long dims[3];
  double spacing[3];
  long long strides[2];  // elements between voxels along axes 0 and 1; 0 = dense
  int label;
  int reserved;
};

// A label's bounding box (inclusive voxel indices; lo = INT_MAX, hi = -1 when
// empty) and voxel count, accumulated by the label pass.
struct LabelAcc {
  int lo[3];
  int hi[3];
  unsigned long long n;
};

// Magic numbers of the kernels' 32-bit division by D (numerators < 2^31):
// floor(n / D) = (n * m) >> sh, sh = 31 + ceil(log2 D), m = floor(2^sh / D) + 1.
__host__ __device__ inline void magic_div(unsigned int D, unsigned int& m, int& sh) {
  int k = 0;
  while ((1ull << k) < D) ++k;
  sh = 31 + k;
  m = (unsigned int)((1ull << sh) / D + 1);
}

// Fills the mesh-pass geometry of a ROI (everything but its brick and bucket
// offsets) and returns its brick count.  Strides of 0 mean a dense layout.
// tz: cube planes per brick (1..kTZ).
__host__ __device__ inline long long roi_fill(Roi& R, const void* vol, const long long dims[3],
                                              const double spacing[3], long long stride0, long long stride1,
                                              int label, int tz = kTZ) {
  R.vol = vol;
  for (int k = 0; k < 3; ++k) {
    R.d[k] = (int)dims[k];
    R.s[k] = spacing[k];
  }
  R.stride1 = stride1 > 0 ? stride1 : (long long)R.d[2];
  R.stride0 = stride0 > 0 ? stride0 : (long long)R.d[1] * R.d[2];
  R.label = label;
  R.status = 0;
  R.tz = tz;
  R.G = (R.d[2] + 1 + 31) / 32;
  R.nrg = (R.d[1] + 1) * R.G;
  R.nzc = (R.d[0] + 1 + tz - 1) / tz;
  R.bpz = (R.nrg + kBrickThreads - 1) / kBrickThreads;
  magic_div((unsigned int)R.G, R.mG, R.shG);
  magic_div((unsigned int)(kBrickThreads + 1 + R.G), R.mNW, R.shNW);
  return (long long)R.nzc * R.bpz;
}

// Plane buckets of a ROI: 2 d_k + 1 per axis.
__host__ __device__ inline long long roi_buckets(const int d[3]) {
  return 2ll * d[0] + 2ll * d[1] + 2ll * d[2] + 3;
}

// Sets the bucket offsets of a ROI whose buckets start at b0.
__host__ __device__ inline void roi_set_buckets(Roi& R, long long b0) {
  R.bucket_base[0] = b0;
  R.bucket_base[1] = b0 + 2ll * R.d[0] + 1;
  R.bucket_base[2] = R.bucket_base[1] + 2ll * R.d[1] + 1;
}

// Per-ROI case data of binary masks in one buffer: 256 case areas (FP64) per
// ROI, then 256 active-cube counts (uint64) per ROI.
__host__ __device__ inline unsigned long long* case_hist(double* case_area, long long n_rois) {
  return reinterpret_cast<unsigned long long*>(case_area + 256 * n_rois);
}
__host__ __device__ inline const unsigned long long* case_hist(const double* case_area, long long n_rois) {
  return reinterpret_cast<const unsigned long long*>(case_area + 256 * n_rois);
}

// Surface area of a binary mask's ROI from its per-case areas and active-cube
// counts: the 256 products n_c a_c summed by a fixed halving tree (so the
// result does not depend on the order in which the cubes were visited).
// Called by threads 0..255 of a workgroup (all of them, or none: it holds
// barriers); s: 256 doubles of shared memory.  The sum is in s[0] afterwards.
__device__ inline void binary_area_tree(const double* area, const unsigned long long* count, double* s) {
  const int c = threadIdx.x;
  if (c < 256) s[c] = count[c] ? __dmul_rn((double)count[c], area[c]) : 0.0;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (c < w) s[c] = __dadd_rn(s[c], s[c + w]);
    __syncthreads();
  }
}

struct BrickPart {
  int nv, nt;
  int bb[6];         // min corner (z, y, x) min / max of active cubes
  double area;       // soft: area partial (binary masks: counted per case instead)
  double vol_d;      // soft: signed volume partial
  long long vol_i;   // binary: signed volume partial in units of s0*s1*s2/48
  // inside-voxel moments in voxel indices (only when the call asks for them):
  // count, sums of z, y, x, of zz, yy, xx, and of zy, zx, yx
  long long mom[10];
  long long stage;   // first row of the brick's vertices in the mesh pass's staging list
};

struct RoiMeta {
  long long V, T;
  long long row_off;  // first layout-0 row
  long long V_pad;    // rows of the 3D segment (0 if V < 2)
  double area;
  double vol;         // signed volume
  double center[3];   // subtracted from positions before rounding to FP32
  double R2;          // bound on |centred FP32 position|^2
  int bb[6];
  long long prune_off;  // first (column, column) pair of the ROI in the pruning pass (pruned ROIs)
  long long n_in;     // inside voxels (when moments are asked for)
  double cov[6];      // covariance of their physical coordinates: zz, yy, xx, zy, zx, yx
};

struct Seg {
  long long row_begin;  // first row (multiple of kBlk)
  int n_rows;           // multiple of kSegAlign
  int group;            // roi * 4 + feature
};

struct Col {
  long long row_begin;  // the segment's first row
  int n_rows;           // the segment's rows
  int group;            // the segment's group (roi * 4 + feature)
  int jc;               // column chunk index within the segment
  int e;                // scale exponent of the ROI's split-f16 operands
};

// 3D pruning: per 32-row block of layout 0, the bounding box of its centred
// FP32 positions and seven packed (value, row) maxima; per ROI, the seven
// seeds and the partners found by two farthest-point sweeps; the pruned work
// items of the 3D pair pass.
struct BlkRec {
  float box[6];                 // lo x, y, z, hi x, y, z
  int pad_[2];
  unsigned long long key[7];    // (ordered float bits << 32) | (0xffffffff - row)
  float tbox[6];                // the box of the row tile starting at this block (tile starts only)
  float cbox[6];                // the box of the 1024-row column starting at this block (column starts only)
};

struct RoiSeed {
  unsigned long long key[3][7];  // 0: seed rows, 1: farthest from each seed, 2: farthest from those
};

struct PItem {
  int rb;      // first 32-row block of the segment
  int nb;      // its 32-row blocks
  int i0;      // first row block of the tile
  int j0, j1;  // column blocks [j0, j1)
  int e;       // scale exponent of the split-f16 operands
  int pad_[2];
};

// Per-group results of the diameter passes.
struct GroupRes {
  unsigned long long best_bits;  // bits of the exact FP64 max squared distance
  unsigned long long id_lo;      // smallest id of the chosen pair
  unsigned long long id_hi;      // larger id of the chosen pair
  int row_i, row_j;              // layout-0 rows of the chosen pair
  float gmax;                    // max over rows of the FP32 row maxima
  int n_cand;
};

}  // namespace s3d
