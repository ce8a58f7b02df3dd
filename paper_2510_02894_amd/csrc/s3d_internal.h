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
constexpr int kCounterWords = kWorkStride * (1 + kWorkParts);  // size of the counter block

// Key of a vertex: edge (u, u + e_a): bits 0..19 u2+1, 20..39 u1+1, 40..59 u0+1, 60..61 a.
__host__ __device__ inline uint64_t pack_key(int u0, int u1, int u2, int a) {
  return (uint64_t)(uint32_t)(u2 + 1) | ((uint64_t)(uint32_t)(u1 + 1) << 20) |
         ((uint64_t)(uint32_t)(u0 + 1) << 40) | ((uint64_t)a << 60);
}

struct Roi {
  const void* vol;        // this ROI's volume (uint8 or float32)
  int d[3];
  int G;                  // row-groups per cube row: ceil((d2 + 1) / 32)
  double s[3];
  long long brick_begin;  // first brick
  int nrg;                // (d1 + 1) * G
  int nzc;                // z-chunks: ceil((d0 + 1) / kTZ)
  int bpz;                // bricks per z-chunk: ceil(nrg / kBrickThreads)
  int shG;                // floor(n / G) = (n * mG) >> shG for 0 <= n < 2^31
  unsigned int mG;
  unsigned int mNW;       // the same for the tile width kBrickThreads + 1 + G
  int shNW;
  int pad_;
  long long bucket_base[3];  // first global plane bucket of each axis
};

struct BrickPart {
  int nv, nt;
  int bb[6];         // min corner (z, y, x) min / max of active cubes
  double area;
  double vol_d;      // soft: signed volume partial
  long long vol_i;   // binary: signed volume partial in units of s0*s1*s2/48
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
  int pad_[2];
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
