// prune.hip -- exact 3D diameter without visiting every vertex pair.
//
// The paper computes the maximum vertex distance by brute force over all
// pairs (Sec. 2, "Parallel diameter calculation").  The maximum itself is all
// that is needed, so a pair whose distance provably stays below a distance
// that some pair reaches can be skipped.  Per ROI with at least `min_v`
// vertices (smaller ROIs stay with the all-pairs work list):
//   1. bounds: every 32-row block of the ROI's vertex rows gets the bounding
//      box of its (centred FP32) positions, and so does every row tile (the
//      pair pass's IT blocks) and every 1024-row column (kPruneSB blocks);
//   2. a lower bound L on the diameter: seven seed vertices (the extremes
//      along +-x, +-y, +-z and the vertex farthest from the box centre), the
//      vertex farthest from each seed, and the vertex farthest from each of
//      those (two farthest-point sweeps); L^2 is the largest squared distance
//      met, i.e. the distance of an actual vertex pair, so L <= D;
//   3. work items: every pair of columns (i <= j) is tested by the largest
//      distance between their boxes; for a pair that can reach
//      thr = L^2 (1 - 2^-10), each row tile of column i is tested against each
//      block of column j (the largest distance between two boxes bounds every
//      pair between them), and each tile with a surviving block becomes one
//      item covering its first to last surviving block.
// The matrix-core pair pass then runs only these items.  Every pair at the
// maximum distance D >= L lies in a surviving item (a column pair's boxes
// contain its tiles' and blocks' boxes, so the coarse test never drops a tile
// that the fine test keeps), so the row maxima of the rows that hold a
// maximising pair, the group maximum, and hence the rows handed to the exact
// FP64 refinement, which rescans them against all vertices, are those of the
// full pass: the result is the exact maximum and the same canonical pair.
// The margin 2^-10 covers the FP32 rounding of positions, boxes and L^2
// (about 2^-20 relative) many times over.
//
// Seed keys are reduced in block-major chunks (one atomic per wave, ROI and
// key), and the column-pair tests run in a persistent grid over all pruned
// ROIs' column pairs.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "s3d_device.h"
#include "s3d_launch.h"

namespace s3d {

namespace {

enum { T_ROWS0 = 0, T_NPAIR = 7 };

// Monotone map of a float to an unsigned int (larger float, larger integer).
__device__ inline unsigned int ord_bits(float v) {
  const unsigned int b = __float_as_uint(v);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ inline float ord_float(unsigned int u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// (value, row) key: the larger value wins, then the smaller row.
__device__ inline unsigned long long vkey(float v, long long row) {
  return ((unsigned long long)ord_bits(v) << 32) | (unsigned long long)(0xffffffffu - (unsigned int)row);
}

__device__ inline long long key_row(unsigned long long k) {
  return (long long)(0xffffffffu - (unsigned int)(k & 0xffffffffull));
}

// Centred FP32 position of a row, from the pair pass's operands: the split-f16
// B operand (h + l, scaled by 2^e) or the FP32 position blocks.
__device__ inline void row_pos(const float* __restrict__ pos, const uint4* __restrict__ posh, long long row, int e,
                               float p[3]) {
  if (posh) {
    const uint4 a = posh[2 * row];
    const v8h h = *(const v8h*)&a;  // h0 h1 h2 l0 l1 l2 h0 h1
#pragma unroll
    for (int c = 0; c < 3; ++c) p[c] = ldexpf((float)h[c] + (float)h[3 + c], -e);
  } else {
    const float* b = pos + (row >> 4) * 64 + (row & 15);
    p[0] = b[0];
    p[1] = b[16];
    p[2] = b[32];
  }
}

// Largest squared distance between a point of box a and a point of box b.
__device__ inline float box_far2(const float* a, const float* b) {
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float d = fmaxf(a[3 + c] - b[c], b[3 + c] - a[c]);
    s += d * d;
  }
  return s;
}

// Whether a ROI's 3D pairs are pruned (else they stay in the all-pairs work list).
__device__ inline bool pruned_roi(const RoiMeta& M, int min_v) { return M.V >= 2 && M.V >= min_v; }

// The ROI of a layout-0 row, and whether it is pruned.
struct RowRoi {
  int roi;
  bool on;
};

__device__ inline RowRoi row_roi(const int* __restrict__ blkseg, const RoiMeta* __restrict__ meta, long long row,
                                 int min_v) {
  RowRoi r;
  r.roi = blkseg[row >> 4];
  r.on = pruned_roi(meta[r.roi], min_v);
  return r;
}

// Rows per lane in the row passes: a 32-row block is held by 4 lanes, so its
// box and keys need two shuffle steps (a wave covers 512 rows).
constexpr int kRowsPerLane = 8;

__device__ inline float quad_min(float v) {
  v = fminf(v, __shfl_xor(v, 1, 64));
  return fminf(v, __shfl_xor(v, 2, 64));
}

__device__ inline float quad_max(float v) {
  v = fmaxf(v, __shfl_xor(v, 1, 64));
  return fmaxf(v, __shfl_xor(v, 2, 64));
}

__device__ inline unsigned long long quad_max_u64(unsigned long long v) {
  unsigned long long o = __shfl_xor(v, 1, 64);
  v = o > v ? o : v;
  o = __shfl_xor(v, 2, 64);
  return o > v ? o : v;
}

// Pass 1: per 32-row block, its box and its seed keys (largest x, y, z, -x,
// -y, -z and |p|^2).  The first row of each pruned ROI also clears its seed
// record (the reduction passes take atomic maxima into it).
__global__ __launch_bounds__(256) void k_prune_box(const float* __restrict__ pos, const uint4* __restrict__ posh,
                                                   const RoiMeta* __restrict__ meta, const int* __restrict__ blkseg,
                                                   const long long* __restrict__ totals, int min_v,
                                                   BlkRec* __restrict__ rec, RoiSeed* __restrict__ seed) {
  const long long rows0 = totals[T_ROWS0];
  const int lane = threadIdx.x & 63;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long base = (((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * (64 * kRowsPerLane);
       base < rows0; base += nwaves * 64 * kRowsPerLane) {
    // four lanes per 32-row block, each taking its rows (lane & 3) + 4 i, so
    // that a load instruction of the wave reads whole cache lines
    const long long blk = base + (long long)(lane >> 2) * 32, r0 = blk + (lane & 3);
    RowRoi rr = {0, false};
    if (blk < rows0) rr = row_roi(blkseg, meta, blk, min_v);  // uniform per block (rows0 is a multiple of 32)
    float box[6] = {3.0e38f, 3.0e38f, 3.0e38f, -3.0e38f, -3.0e38f, -3.0e38f};
    unsigned long long key[7] = {0ull, 0ull, 0ull, 0ull, 0ull, 0ull, 0ull};
    if (rr.on) {
      const RoiMeta& M = meta[rr.roi];
      const int e = h_scale_exp(M.R2);
      if (blk == M.row_off && (lane & 3) == 0) {
        for (int q = 0; q < 3; ++q)
          for (int c = 0; c < 7; ++c) seed[rr.roi].key[q][c] = 0ull;
      }
      float p[kRowsPerLane][3];
#pragma unroll
      for (int i = 0; i < kRowsPerLane; ++i) row_pos(pos, posh, r0 + 4 * i, e, p[i]);
#pragma unroll
      for (int i = 0; i < kRowsPerLane; ++i) {
        const float val[7] = {p[i][0], p[i][1], p[i][2], -p[i][0], -p[i][1], -p[i][2],
                              p[i][0] * p[i][0] + p[i][1] * p[i][1] + p[i][2] * p[i][2]};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          box[c] = fminf(box[c], p[i][c]);
          box[3 + c] = fmaxf(box[3 + c], p[i][c]);
        }
#pragma unroll
        for (int c = 0; c < 7; ++c) {
          const unsigned long long k = vkey(val[c], r0 + 4 * i);
          key[c] = k > key[c] ? k : key[c];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      box[c] = quad_min(box[c]);
      box[3 + c] = quad_max(box[3 + c]);
    }
#pragma unroll
    for (int c = 0; c < 7; ++c) key[c] = quad_max_u64(key[c]);
    if (rr.on && (lane & 3) == 0) {
      BlkRec& R = rec[blk >> 5];
#pragma unroll
      for (int c = 0; c < 6; ++c) R.box[c] = box[c];
#pragma unroll
      for (int c = 0; c < 7; ++c) R.key[c] = key[c];
    }
  }
}

// Passes 2, 4, 6: the maxima of the blocks' keys per ROI into seed slot
// `slot`.  A wave walks a contiguous range of blocks, 64 kRedPerLane at a time
// (kRedPerLane per lane, their loads issued together); each lane keeps the
// maxima of its blocks per ROI, and the lanes that end on the same ROI combine
// theirs into the wave's maxima of its last ROI.  With BOXES (pass 2) the lanes
// also write the box of every row tile (it_blocks blocks) and every column
// (kPruneSB blocks) that starts among their blocks.
constexpr int kRedPerLane = 4;

__device__ inline void seed_max(RoiSeed* seed, int roi, int slot, const unsigned long long* k) {
#pragma unroll
  for (int c = 0; c < 7; ++c)
    if (k[c]) atomicMax(&seed[roi].key[slot][c], k[c]);
}

// Box of blocks [b, b + n) of a ROI's rows (n <= kPruneSB), eight blocks'
// loads in flight at a time.
__device__ inline void blocks_box(const BlkRec* __restrict__ rec, long long b, int n, float* bx) {
  for (int u0 = 0; u0 < n; u0 += 8) {
    float lo[8][3], hi[8][3];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const long long bb = b + min(u0 + u, n - 1);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        lo[u][c] = rec[bb].box[c];
        hi[u][c] = rec[bb].box[3 + c];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        bx[c] = fminf(bx[c], lo[u][c]);
        bx[3 + c] = fmaxf(bx[3 + c], hi[u][c]);
      }
  }
}

template <bool BOXES>
__global__ __launch_bounds__(256) void k_prune_reduce(BlkRec* __restrict__ rec, const RoiMeta* __restrict__ meta,
                                                      const int* __restrict__ blkseg,
                                                      const long long* __restrict__ totals, int min_v,
                                                      RoiSeed* __restrict__ seed, int slot, int it_blocks) {
  const long long nblk = totals[T_ROWS0] / 32;
  const int lane = threadIdx.x & 63;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  // a contiguous range of blocks per wave, so that its iterations mostly meet
  // the same ROI: the wave keeps the maxima of the last ROI it met (wroi,
  // wk) and issues atomics only when the ROI changes
  constexpr long long kStep = 64 * kRedPerLane;
  const long long per = (nblk + nwaves - 1) / nwaves;
  const long long w0 = wave * ((per + kStep - 1) / kStep * kStep);
  const long long w1 = min(w0 + (per + kStep - 1) / kStep * kStep, nblk);
  int wroi = -1;
  unsigned long long wk[7] = {0ull, 0ull, 0ull, 0ull, 0ull, 0ull, 0ull};
  for (long long base = w0; base < w1; base += kStep) {
    const long long b0 = base + (long long)lane * kRedPerLane;
    int roiq[kRedPerLane];
    unsigned long long kq[kRedPerLane][7];
#pragma unroll
    for (int q = 0; q < kRedPerLane; ++q) {
      const long long blk = min(b0 + q, nblk - 1);
      roiq[q] = blkseg[2 * blk];
#pragma unroll
      for (int c = 0; c < 7; ++c) kq[q][c] = rec[blk].key[c];
    }
    int cur = -1;
    unsigned long long k[7] = {0ull, 0ull, 0ull, 0ull, 0ull, 0ull, 0ull};
#pragma unroll
    for (int q = 0; q < kRedPerLane; ++q) {
      const long long blk = b0 + q;
      if (blk >= w1) break;
      const int roi = roiq[q];
      const RoiMeta& M = meta[roi];
      if (!pruned_roi(M, min_v)) continue;
      if (roi != cur) {
        if (cur >= 0) seed_max(seed, cur, slot, k);
        cur = roi;
#pragma unroll
        for (int c = 0; c < 7; ++c) k[c] = 0ull;
      }
#pragma unroll
      for (int c = 0; c < 7; ++c) k[c] = kq[q][c] > k[c] ? kq[q][c] : k[c];
      if (BOXES) {
        const long long rb = M.row_off / 32;
        const int nb = (int)(M.V_pad / 32), rel = (int)(blk - rb);
        if (rel % it_blocks == 0 || rel % kPruneSB == 0) {
          float tb[6] = {3.0e38f, 3.0e38f, 3.0e38f, -3.0e38f, -3.0e38f, -3.0e38f};
          blocks_box(rec, blk, min(it_blocks, nb - rel), tb);
          if (rel % it_blocks == 0)
            for (int c = 0; c < 6; ++c) rec[blk].tbox[c] = tb[c];
          if (rel % kPruneSB == 0) {
            // the column box also covers the tile's blocks
            float cb[6] = {tb[0], tb[1], tb[2], tb[3], tb[4], tb[5]};
            if (nb - rel > it_blocks) blocks_box(rec, blk + it_blocks, min(kPruneSB, nb - rel) - it_blocks, cb);
            for (int c = 0; c < 6; ++c) rec[blk].cbox[c] = cb[c];
          }
        }
      }
    }
    // lanes ending on the same ROI combine their maxima into the wave's
    unsigned long long todo = __ballot(cur >= 0);
    while (todo) {
      const int leader = __ffsll((long long)todo) - 1;
      const int gl = __shfl(cur, leader, 64);
      const unsigned long long same = __ballot(cur == gl) & todo;
      unsigned long long v[7];
#pragma unroll
      for (int c = 0; c < 7; ++c) {
        v[c] = cur == gl ? k[c] : 0ull;
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) {
          const unsigned long long o = __shfl_xor(v[c], m, 64);
          v[c] = o > v[c] ? o : v[c];
        }
      }
      if (gl != wroi) {
        if (wroi >= 0 && lane == 0) seed_max(seed, wroi, slot, wk);
        wroi = gl;
#pragma unroll
        for (int c = 0; c < 7; ++c) wk[c] = 0ull;
      }
#pragma unroll
      for (int c = 0; c < 7; ++c) wk[c] = v[c] > wk[c] ? v[c] : wk[c];
      todo &= ~same;
    }
  }
  // the waves' last ROIs: one atomic per key and ROI for the workgroup
  __shared__ int s_roi[4];
  __shared__ unsigned long long s_key[4][7];
  const int wid = threadIdx.x >> 6;
  if (lane == 0) {
    s_roi[wid] = wroi;
#pragma unroll
    for (int c = 0; c < 7; ++c) s_key[wid][c] = wk[c];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 0; w < 4; ++w) {
      const int r = s_roi[w];
      if (r < 0) continue;
      unsigned long long v[7];
#pragma unroll
      for (int c = 0; c < 7; ++c) v[c] = s_key[w][c];
      for (int w2 = w + 1; w2 < 4; ++w2) {
        if (s_roi[w2] != r) continue;
#pragma unroll
        for (int c = 0; c < 7; ++c) v[c] = s_key[w2][c] > v[c] ? s_key[w2][c] : v[c];
        s_roi[w2] = -1;
      }
      seed_max(seed, r, slot, v);
    }
  }
}

// Threshold of the tile test for ROI r: L^2 (1 - 2^-10), L^2 the largest
// squared distance the two farthest-point sweeps met (seed slots 1 and 2).
__device__ inline float prune_threshold(const RoiSeed* __restrict__ seed, int r) {
  float L2 = 0.0f;
#pragma unroll
  for (int q = 1; q < 3; ++q)
#pragma unroll
    for (int c = 0; c < 7; ++c) L2 = fmaxf(L2, ord_float((unsigned int)(seed[r].key[q][c] >> 32)));
  return L2 * (1.0f - 0.0009765625f);
}

// Passes 3, 5: per block, the packed maxima over its rows of the squared
// distance to each of the seven vertices in seed slot `src` of its ROI.
__global__ __launch_bounds__(256) void k_prune_far(const float* __restrict__ pos, const uint4* __restrict__ posh,
                                                   const RoiMeta* __restrict__ meta, const int* __restrict__ blkseg,
                                                   const long long* __restrict__ totals, int min_v,
                                                   const RoiSeed* __restrict__ seed, int src,
                                                   BlkRec* __restrict__ rec) {
  const long long rows0 = totals[T_ROWS0];
  const int lane = threadIdx.x & 63;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long base = (((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * (64 * kRowsPerLane);
       base < rows0; base += nwaves * 64 * kRowsPerLane) {
    const long long blk = base + (long long)(lane >> 2) * 32, r0 = blk + (lane & 3);  // as in k_prune_box
    RowRoi rr = {0, false};
    if (blk < rows0) rr = row_roi(blkseg, meta, blk, min_v);
    unsigned long long key[7] = {0ull, 0ull, 0ull, 0ull, 0ull, 0ull, 0ull};
    if (rr.on) {
      const int e = h_scale_exp(meta[rr.roi].R2);
      float q[7][3];
#pragma unroll
      for (int c = 0; c < 7; ++c) row_pos(pos, posh, key_row(seed[rr.roi].key[src][c]), e, q[c]);
      float p[kRowsPerLane][3];
#pragma unroll
      for (int i = 0; i < kRowsPerLane; ++i) row_pos(pos, posh, r0 + 4 * i, e, p[i]);
#pragma unroll
      for (int i = 0; i < kRowsPerLane; ++i)
#pragma unroll
        for (int c = 0; c < 7; ++c) {
          const float dx = p[i][0] - q[c][0], dy = p[i][1] - q[c][1], dz = p[i][2] - q[c][2];
          const unsigned long long k = vkey(dx * dx + dy * dy + dz * dz, r0 + 4 * i);
          key[c] = k > key[c] ? k : key[c];
        }
    }
#pragma unroll
    for (int c = 0; c < 7; ++c) key[c] = quad_max_u64(key[c]);
    if (rr.on && (lane & 3) == 0) {
#pragma unroll
      for (int c = 0; c < 7; ++c) rec[blk >> 5].key[c] = key[c];
    }
  }
}

// A wave's staging buffer for work items in LDS: items are collected there
// and appended to the global list 64 at a time with one atomic, so that the
// many waves that emit a few items each do not all contend for the list's
// counter.  Every lane of the wave must call push and flush alike.
struct ItemStage {
  PItem* buf;  // this wave's 64 LDS slots
  int n;       // wave-uniform count of staged items

  __device__ void flush(int lane, PItem* __restrict__ items, long long cap, unsigned int* __restrict__ counters) {
    if (n == 0) return;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    unsigned int first = 0;
    if (lane == 0) first = atomicAdd(&counters[3], (unsigned int)n);
    first = __shfl(first, 0, 64);
    for (int i = lane; i < n; i += 64) {
      const long long slot = (long long)first + i;
      if (slot < cap)
        items[slot] = buf[i];
      else
        counters[4] = 1u;  // the list is incomplete: the pruned ROIs' 3D pairs run unpruned
    }
    __builtin_amdgcn_wave_barrier();
    n = 0;
  }
  // Stages the item of every lane with `emit` set (at most 32 per call).
  __device__ void push(bool emit, const PItem& P, int lane, PItem* __restrict__ items, long long cap,
                       unsigned int* __restrict__ counters) {
    const unsigned long long em = __ballot(emit);
    const int k = __popcll(em);
    if (k == 0) return;
    if (n + k > 64) flush(lane, items, cap, counters);
    if (emit) buf[n + __popcll(em & ((1ull << lane) - 1ull))] = P;
    n += k;
  }
};

// Pass 7: the work items.  A persistent grid runs over the column pairs
// (i, j) of all pruned ROIs (ROI r owns ncol^2 consecutive indices from
// meta[r].prune_off; pairs with i > j are skipped): each lane tests one
// column pair by its columns' boxes, then every surviving pair is expanded by
// the whole wave: lane l tests row tile l / LPT of column i against LPT
// consecutive blocks of column j, and each tile with a surviving block
// becomes an item over its first to last surviving block.
template <int IT>
__global__ __launch_bounds__(256) void k_prune_items(const BlkRec* __restrict__ rec, const RoiMeta* __restrict__ meta,
                                                     int n_rois, const long long* __restrict__ totals,
                                                     const RoiSeed* __restrict__ seed, PItem* __restrict__ items,
                                                     long long cap, unsigned int* __restrict__ counters) {
  constexpr int TPC = kPruneSB / IT;   // row tiles per column
  constexpr int LPT = 64 / TPC;        // lanes per tile
  constexpr int BPL = kPruneSB / LPT;  // column blocks per lane
  static_assert(TPC * IT == kPruneSB && LPT * TPC == 64 && BPL * LPT == kPruneSB, "tile and wave shapes");
  const long long total = totals[T_NPAIR];
  const int lane = threadIdx.x & 63;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  int thr_roi = -1;
  float thr_val = 0.0f;
  __shared__ PItem s_stage[4][64];
  ItemStage stage{s_stage[threadIdx.x >> 6], 0};
  for (long long base = (((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 64; base < total;
       base += nwaves * 64) {
    const long long idx = base + lane;
    bool pass = false;
    int r = 0, ci = 0, cj = 0;
    float thr_r = 0.0f;
    if (idx < total) {
      int lo = 0, hi = n_rois - 1;  // the last ROI whose first column pair is <= idx
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (meta[mid].prune_off <= idx)
          lo = mid;
        else
          hi = mid - 1;
      }
      r = lo;
      const RoiMeta& M = meta[r];
      const int nb = (int)(M.V_pad / 32);
      const int ncol = (nb + kPruneSB - 1) / kPruneSB;
      const long long local = idx - M.prune_off;
      ci = (int)(local / ncol);
      cj = (int)(local - (long long)ci * ncol);
      if (ci <= cj) {
        if (r != thr_roi) {  // the threshold of the lane's last ROI is kept
          thr_roi = r;
          thr_val = prune_threshold(seed, r);
        }
        thr_r = thr_val;
        const long long rb = M.row_off / 32;
        pass = box_far2(rec[rb + ci * kPruneSB].cbox, rec[rb + cj * kPruneSB].cbox) >= thr_r;
      }
    }
    // Surviving column pairs, two at a time: the box loads of both are issued
    // before either is tested (one memory round trip per two pairs).
    unsigned long long todo = __ballot(pass);
    while (todo) {
      int srcl[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        srcl[u] = todo ? __ffsll((long long)todo) - 1 : -1;
        if (todo) todo &= todo - 1ull;
      }
      const int t = lane / LPT, g = lane % LPT;
      float tb[2][6], jbx[2][BPL][6];
      int nb[2], rb[2], i0[2], j[2];
      float thr[2];
      double r2[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        nb[u] = 0;
        rb[u] = 0;
        i0[u] = 0;
        j[u] = 0;
        thr[u] = 0.0f;
        r2[u] = 0.0;
        if (srcl[u] < 0) continue;  // uniform over the wave
        const int rr = __shfl(r, srcl[u], 64), i = __shfl(ci, srcl[u], 64);
        j[u] = __shfl(cj, srcl[u], 64);
        thr[u] = __shfl(thr_r, srcl[u], 64);
        const RoiMeta& M = meta[rr];
        nb[u] = (int)(M.V_pad / 32);
        rb[u] = (int)(M.row_off / 32);
        r2[u] = M.R2;
        i0[u] = i * kPruneSB + t * IT;  // the tile's first block
        const int jb0 = j[u] * kPruneSB + g * BPL;  // this lane's first block of column j
        const int ic = min(i0[u], nb[u] - 1);
#pragma unroll
        for (int c = 0; c < 6; ++c) tb[u][c] = rec[rb[u] + ic].tbox[c];
#pragma unroll
        for (int q = 0; q < BPL; ++q) {
          const int jj = min(jb0 + q, nb[u] - 1);
#pragma unroll
          for (int c = 0; c < 6; ++c) jbx[u][q][c] = rec[rb[u] + jj].box[c];
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (srcl[u] < 0) continue;
        const int jb0 = j[u] * kPruneSB + g * BPL;
        unsigned int bits = 0u;  // surviving blocks of column j (bit = block - j * kPruneSB)
        if (i0[u] < nb[u]) {
#pragma unroll
          for (int q = 0; q < BPL; ++q) {
            const int jj = jb0 + q;
            if (jj < nb[u] && jj >= i0[u] && box_far2(tb[u], jbx[u][q]) >= thr[u]) bits |= 1u << (g * BPL + q);
          }
        }
#pragma unroll
        for (int m = 1; m < LPT; m <<= 1) bits |= __shfl_xor(bits, m, 64);
        PItem P;
        P.rb = rb[u];
        P.nb = nb[u];
        P.i0 = i0[u];
        P.j0 = j[u] * kPruneSB + (bits ? __ffs(bits) - 1 : 0);
        P.j1 = j[u] * kPruneSB + (32 - __clz(bits));
        P.e = h_scale_exp(r2[u]);
        P.pad_[0] = P.pad_[1] = 0;
        stage.push(g == 0 && bits != 0u, P, lane, items, cap, counters);
      }
    }
  }
  stage.flush(lane, items, cap, counters);
}

unsigned grid_rows(long long n, long long cap = 4096) {
  long long g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

hipError_t launch_prune(const PairBufs& B, hipStream_t st) {
  const float* pos = B.tune.kernel == 1 ? nullptr : B.pos;
  const uint4* posh = B.tune.kernel == 1 ? B.posh : nullptr;
  const int it_blocks = B.tune.itile == 8 ? 4 : 2;
  const unsigned g = grid_rows((B.rows0 + kRowsPerLane - 1) / kRowsPerLane);
  const unsigned gb = grid_rows((B.rows0 / 32 + kRedPerLane - 1) / kRedPerLane + 1, 1024);
  hipLaunchKernelGGL(k_prune_box, dim3(g), dim3(256), 0, st, pos, posh, B.meta, B.blkseg, B.totals, B.prune_min_v,
                     B.blkrec, B.rseed);
  hipLaunchKernelGGL(k_prune_reduce<true>, dim3(gb), dim3(256), 0, st, B.blkrec, B.meta, B.blkseg, B.totals,
                     B.prune_min_v, B.rseed, 0, it_blocks);
  for (int s = 1; s < 3; ++s) {
    hipLaunchKernelGGL(k_prune_far, dim3(g), dim3(256), 0, st, pos, posh, B.meta, B.blkseg, B.totals, B.prune_min_v,
                       B.rseed, s - 1, B.blkrec);
    hipLaunchKernelGGL(k_prune_reduce<false>, dim3(gb), dim3(256), 0, st, B.blkrec, B.meta, B.blkseg, B.totals,
                       B.prune_min_v, B.rseed, s, it_blocks);
  }
  // a persistent grid over the column pairs (their count is known on the device only)
  const unsigned gi = (unsigned)std::max(1, B.cu_count * 8);
  if (it_blocks == 4)
    hipLaunchKernelGGL(k_prune_items<4>, dim3(gi), dim3(256), 0, st, B.blkrec, B.meta, B.n_rois, B.totals, B.rseed,
                       B.pitems, B.pitem_cap, B.counters);
  else
    hipLaunchKernelGGL(k_prune_items<2>, dim3(gi), dim3(256), 0, st, B.blkrec, B.meta, B.n_rois, B.totals, B.rseed,
                       B.pitems, B.pitem_cap, B.counters);
  return hipGetLastError();
}

}  // namespace s3d
