// prune.hip -- exact 3D diameter without visiting every vertex pair.
//
// The paper computes the maximum vertex distance by brute force over all
// pairs (Sec. 2, "Parallel diameter calculation").  The maximum itself is all
// that is needed, so a pair whose distance provably stays below a distance
// that some pair reaches can be skipped.  Per ROI:
//   1. bounds: every 32-row block of the ROI's vertex rows gets the bounding
//      box of its (centred FP32) positions;
//   2. a lower bound L on the diameter: seven seed vertices (the extremes
//      along +-x, +-y, +-z and the vertex farthest from the box centre), the
//      vertex farthest from each seed, and the vertex farthest from each of
//      those (two farthest-point sweeps); L^2 is the largest squared distance
//      met, i.e. the distance of an actual vertex pair, so L <= D;
//   3. work items: for each row tile (IT blocks) and each column of 32 blocks
//      of the upper triangle, the tile's box is tested against the column's
//      box, then against each block's box; the largest distance between two
//      boxes bounds every pair between them, and tiles whose bound is below
//      L^2 (1 - 2^-10) are dropped.  Each surviving (tile, column) becomes
//      one item covering its first to last surviving block.
// The matrix-core pair pass then runs only these items.  Every pair at the
// maximum distance D >= L lies in a surviving item, so the row maxima of the
// rows that hold a maximising pair, the group maximum, and hence the rows
// handed to the exact FP64 refinement, which rescans them against all vertices,
// are those of the full pass: the result is the exact maximum and the same
// canonical pair.  The margin 2^-10 covers the FP32 rounding of positions,
// boxes and L^2 (about 2^-20 relative) many times over.
#include <hip/hip_runtime.h>

#include "s3d_device.h"
#include "s3d_launch.h"

namespace s3d {

namespace {

enum { T_ROWS0 = 0, T_NSB = 7 };

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

// Maximum over the 32 lanes of a half wave.
__device__ inline float half_max(float v) {
#pragma unroll
  for (int m = 1; m < 32; m <<= 1) v = fmaxf(v, __shfl_xor(v, m, 64));
  return v;
}

__device__ inline float half_min(float v) {
#pragma unroll
  for (int m = 1; m < 32; m <<= 1) v = fminf(v, __shfl_xor(v, m, 64));
  return v;
}

__device__ inline unsigned long long half_max_u64(unsigned long long v) {
#pragma unroll
  for (int m = 1; m < 32; m <<= 1) {
    const unsigned long long o = __shfl_xor(v, m, 64);
    v = o > v ? o : v;
  }
  return v;
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

// The ROI of a layout-0 row, and whether its 3D segment has pairs.
struct RowRoi {
  int roi;
  bool on;
};

__device__ inline RowRoi row_roi(const int* __restrict__ blkseg, const RoiMeta* __restrict__ meta, long long row) {
  RowRoi r;
  r.roi = blkseg[row >> 4];
  r.on = meta[r.roi].V >= 2;
  return r;
}

// Pass 1: per 32-row block, its box and its seed keys (largest x, y, z, -x,
// -y, -z and |p|^2).  The first row of each ROI also clears its seed record.
__global__ __launch_bounds__(256) void k_prune_box(const float* __restrict__ pos, const uint4* __restrict__ posh,
                                                   const RoiMeta* __restrict__ meta, const int* __restrict__ blkseg,
                                                   const long long* __restrict__ totals, BlkRec* __restrict__ rec,
                                                   RoiSeed* __restrict__ seed) {
  const long long rows0 = totals[T_ROWS0];
  const int lane = threadIdx.x & 63;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long base = (((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 64; base < rows0;
       base += nwaves * 64) {
    const long long row = base + lane;
    const bool valid = row < rows0;  // uniform per half wave (rows0 is a multiple of 32)
    RowRoi rr = {0, false};
    if (valid) rr = row_roi(blkseg, meta, row);
    float p[3] = {0.0f, 0.0f, 0.0f};
    if (rr.on) {
      const RoiMeta& M = meta[rr.roi];
      row_pos(pos, posh, row, h_scale_exp(M.R2), p);
      if (row == M.row_off) {
        RoiSeed z;
        for (int s = 0; s < 3; ++s)
          for (int c = 0; c < 7; ++c) z.key[s][c] = 0ull;
        seed[rr.roi] = z;
      }
    }
    float box[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      box[c] = half_min(rr.on ? p[c] : 3.0e38f);
      box[3 + c] = half_max(rr.on ? p[c] : -3.0e38f);
    }
    const float val[7] = {p[0], p[1], p[2], -p[0], -p[1], -p[2], p[0] * p[0] + p[1] * p[1] + p[2] * p[2]};
    unsigned long long key[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) key[c] = half_max_u64(rr.on ? vkey(val[c], row) : 0ull);
    if (rr.on && (lane & 31) == 0) {
      BlkRec R;
#pragma unroll
      for (int c = 0; c < 6; ++c) R.box[c] = box[c];
      R.pad_[0] = R.pad_[1] = 0;
#pragma unroll
      for (int c = 0; c < 7; ++c) R.key[c] = key[c];
      rec[row >> 5] = R;
    }
  }
}

// Passes 2, 4, 6: per ROI, the maximum of each block key into seed slot
// `slot`.  A wave takes 64 consecutive blocks and issues one atomic per key
// and per distinct ROI among them (usually one).
__global__ __launch_bounds__(256) void k_prune_reduce(const BlkRec* __restrict__ rec, const RoiMeta* __restrict__ meta,
                                                      const int* __restrict__ blkseg,
                                                      const long long* __restrict__ totals, RoiSeed* __restrict__ seed,
                                                      int slot) {
  const long long nblk = totals[T_ROWS0] / 32;
  const int lane = threadIdx.x & 63;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long base = (((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 64; base < nblk;
       base += nwaves * 64) {
    const long long blk = base + lane;
    int g = -1;
    if (blk < nblk) {
      const RowRoi rr = row_roi(blkseg, meta, blk * 32);
      if (rr.on) g = rr.roi;
    }
    unsigned long long todo = __ballot(g >= 0);
    while (todo) {
      const int leader = __ffsll((long long)todo) - 1;
      const int gl = __shfl(g, leader, 64);
      const unsigned long long same = __ballot(g == gl) & todo;
#pragma unroll
      for (int c = 0; c < 7; ++c) {
        unsigned long long v = g == gl ? rec[blk].key[c] : 0ull;
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) {
          const unsigned long long o = __shfl_xor(v, m, 64);
          v = o > v ? o : v;
        }
        if (lane == leader) atomicMax(&seed[gl].key[slot][c], v);
      }
      todo &= ~same;
    }
  }
}

// Passes 3, 5: per block, the packed maxima over its rows of the squared
// distance to each of the seven vertices in seed slot `src` of its ROI.
__global__ __launch_bounds__(256) void k_prune_far(const float* __restrict__ pos, const uint4* __restrict__ posh,
                                                   const RoiMeta* __restrict__ meta, const int* __restrict__ blkseg,
                                                   const long long* __restrict__ totals,
                                                   const RoiSeed* __restrict__ seed, int src,
                                                   BlkRec* __restrict__ rec) {
  const long long rows0 = totals[T_ROWS0];
  const int lane = threadIdx.x & 63;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long base = (((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 64; base < rows0;
       base += nwaves * 64) {
    const long long row = base + lane;
    RowRoi rr = {0, false};
    if (row < rows0) rr = row_roi(blkseg, meta, row);
    unsigned long long key[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) key[c] = 0ull;
    if (rr.on) {
      const int e = h_scale_exp(meta[rr.roi].R2);
      float p[3];
      row_pos(pos, posh, row, e, p);
#pragma unroll
      for (int c = 0; c < 7; ++c) {
        float q[3];
        row_pos(pos, posh, key_row(seed[rr.roi].key[src][c]), e, q);
        const float dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
        key[c] = vkey(dx * dx + dy * dy + dz * dz, row);
      }
    }
#pragma unroll
    for (int c = 0; c < 7; ++c) key[c] = half_max_u64(key[c]);
    if (rr.on && (lane & 31) == 0) {
#pragma unroll
      for (int c = 0; c < 7; ++c) rec[row >> 5].key[c] = key[c];
    }
  }
}

// Pass 7: one wave per (ROI, column of kPruneSB blocks); lanes run over the
// row tiles of the upper triangle that start before the column ends.
template <int IT>
__global__ __launch_bounds__(256) void k_prune_items(const BlkRec* __restrict__ rec, const RoiMeta* __restrict__ meta,
                                                     int n_rois, const long long* __restrict__ totals,
                                                     const RoiSeed* __restrict__ seed, PItem* __restrict__ items,
                                                     long long cap, unsigned int* __restrict__ counters) {
  const int lane = threadIdx.x & 63;
  const long long w = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (w >= totals[T_NSB]) return;  // whole waves leave; the kernel has no barrier
  int lo = 0, hi = n_rois - 1;     // the last ROI whose first column is <= w
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (meta[mid].sb_off <= w)
      lo = mid;
    else
      hi = mid - 1;
  }
  const RoiMeta& M = meta[lo];
  const int nb = (int)(M.V_pad / 32);
  const long long rb = M.row_off / 32;
  const int c0 = (int)(w - M.sb_off) * kPruneSB;
  const int c1 = min(c0 + kPruneSB, nb);
  const int e = h_scale_exp(M.R2);
  float L2 = 0.0f;
  for (int s = 1; s < 3; ++s)
    for (int c = 0; c < 7; ++c) L2 = fmaxf(L2, ord_float((unsigned int)(seed[lo].key[s][c] >> 32)));
  const float thr = L2 * (1.0f - 0.0009765625f);  // 1 - 2^-10
  // the column's box (its blocks' boxes are read again, from cache, by the
  // tiles that pass the column test)
  float cb[6];
  {
    float b[6] = {3.0e38f, 3.0e38f, 3.0e38f, -3.0e38f, -3.0e38f, -3.0e38f};
    if (lane < c1 - c0) {
      const BlkRec& R = rec[rb + c0 + lane];
#pragma unroll
      for (int c = 0; c < 6; ++c) b[c] = R.box[c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float mn = b[c], mx = b[3 + c];
#pragma unroll
      for (int m = 1; m < 64; m <<= 1) {
        mn = fminf(mn, __shfl_xor(mn, m, 64));
        mx = fmaxf(mx, __shfl_xor(mx, m, 64));
      }
      cb[c] = mn;
      cb[3 + c] = mx;
    }
  }
  const int ntile = min((c1 + IT - 1) / IT, (nb + IT - 1) / IT);  // tiles with i0 < c1
  for (int t0 = 0; t0 < ntile; t0 += 64) {
    const int t = t0 + lane;
    int jf = -1, jl = -1;
    const int i0 = t * IT;
    if (t < ntile) {
      float tb[6] = {3.0e38f, 3.0e38f, 3.0e38f, -3.0e38f, -3.0e38f, -3.0e38f};
      for (int r = 0; r < IT && i0 + r < nb; ++r) {
        const BlkRec& R = rec[rb + i0 + r];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          tb[c] = fminf(tb[c], R.box[c]);
          tb[3 + c] = fmaxf(tb[3 + c], R.box[3 + c]);
        }
      }
      if (box_far2(tb, cb) >= thr) {
        for (int j = max(c0, i0); j < c1; ++j)
          if (box_far2(tb, rec[rb + j].box) >= thr) {
            if (jf < 0) jf = j;
            jl = j;
          }
      }
    }
    const bool emit = jf >= 0;
    const unsigned long long m = __ballot(emit);
    if (!m) continue;
    unsigned int first = 0;
    if (lane == 0) first = atomicAdd(&counters[3], (unsigned int)__popcll(m));
    first = __shfl(first, 0, 64);
    if (emit) {
      const long long idx = (long long)first + __popcll(m & ((1ull << lane) - 1ull));
      if (idx < cap) {
        PItem P;
        P.rb = (int)rb;
        P.nb = nb;
        P.i0 = i0;
        P.j0 = jf;
        P.j1 = jl + 1;
        P.e = e;
        P.pad_[0] = P.pad_[1] = 0;
        items[idx] = P;
      } else {
        counters[4] = 1u;  // the list is incomplete: the 3D pairs run unpruned
      }
    }
  }
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
  const unsigned g = grid_rows(B.rows0);
  hipLaunchKernelGGL(k_prune_box, dim3(g), dim3(256), 0, st, pos, posh, B.meta, B.blkseg, B.totals, B.blkrec, B.rseed);
  const unsigned gb = grid_rows(B.rows0 / 32 + 1, 1024);
  hipLaunchKernelGGL(k_prune_reduce, dim3(gb), dim3(256), 0, st, B.blkrec, B.meta, B.blkseg, B.totals, B.rseed, 0);
  for (int s = 1; s < 3; ++s) {
    hipLaunchKernelGGL(k_prune_far, dim3(g), dim3(256), 0, st, pos, posh, B.meta, B.blkseg, B.totals, B.rseed, s - 1,
                       B.blkrec);
    hipLaunchKernelGGL(k_prune_reduce, dim3(gb), dim3(256), 0, st, B.blkrec, B.meta, B.blkseg, B.totals, B.rseed, s);
  }
  // waves: at most one column per 1024 rows plus one partial column per ROI
  const long long waves = B.rows0 / (kPruneSB * 32) + B.n_rois + 1;
  const unsigned gi = (unsigned)((waves + 3) / 4);
  if (B.tune.itile == 8)
    hipLaunchKernelGGL(k_prune_items<4>, dim3(gi), dim3(256), 0, st, B.blkrec, B.meta, B.n_rois, B.totals, B.rseed,
                       B.pitems, B.pitem_cap, B.counters);
  else
    hipLaunchKernelGGL(k_prune_items<2>, dim3(gi), dim3(256), 0, st, B.blkrec, B.meta, B.n_rois, B.totals, B.rseed,
                       B.pitems, B.pitem_cap, B.counters);
  return hipGetLastError();
}

}  // namespace s3d
