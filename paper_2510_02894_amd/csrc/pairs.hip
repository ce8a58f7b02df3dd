// pairs.hip -- maximum vertex distances (paper Sec. 2, "Parallel diameter
// calculation"): the 3D diameter over all vertex pairs and the planar
// diameters over vertex pairs that share a plane of each axis.
//
// Design for CDNA4:
//   * plane buckets by a counting sort on the plane key 2*u_k + [a == k];
//     every bucket with two or more vertices becomes a segment, as does each
//     ROI's whole vertex list, and all segments are processed in one launch;
//   * squared distances come from the Gram form
//       d2(i, j) = w_i + w_j - 2 p_i . p_j,  w = |p|^2,
//     which is a K = 4 contraction [-2x_i, -2y_i, -2z_i, 1] . [x_j, y_j, z_j, w_j]
//     and maps exactly onto v_mfma_f32_16x16x4_f32: one instruction gives the
//     256 pair values of a 16 x 16 tile; the VALU keeps per-row running maxima
//     (v_max3) beside the matrix core;
//   * a wave owns a tile of row blocks (kept in registers as A operands) and
//     streams the column blocks of one column chunk of the upper triangle;
//     work items, in column-major order, are handed out by one atomic counter
//     per XCD over a contiguous range each, so the waves of an XCD share the
//     column data in its L2;
//   * FP32 row maxima are then refined exactly: every row whose FP32 maximum
//     lies within a rigorous rounding bound of the group maximum is rescanned
//     against its whole segment in FP64 (the same operations as the oracle),
//     which yields the exact maximum and the canonical tie-break.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "s3d_device.h"
#include "s3d_launch.h"

namespace s3d {

typedef float v4f __attribute__((ext_vector_type(4)));

enum { T_ROWS0 = 0, T_VMAX = 1, T_ROWS2D = 2, T_NSEG2D = 3, T_NCOL = 4, T_NITEM = 5, T_NEXACT = 6, T_NSB = 7 };

// ---------------------------------------------------------------------------
// Plane buckets.

// Adds 1 to counter[b] for every active lane.  Lanes with the same b form one
// group served by one atomic of its leader; the groups are found first (ALU
// only) and then all leaders issue their atomics together.  (Per-lane atomics
// are slower: lanes of a wave often share a bucket, and colliding atomics
// serialise in memory.)
__device__ inline void wave_aggregated_inc(unsigned int* counter, long long b) {
  unsigned long long todo = __ballot(1);
  const int lane = threadIdx.x & 63;
  unsigned int group = 0;
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const long long bl = __shfl(b, leader, 64);
    const unsigned long long same = __ballot(b == bl) & todo;
    if (lane == leader) group = (unsigned int)__popcll(same);
    todo &= ~same;
  }
  if (group) atomicAdd(&counter[b], group);
}

// As wave_aggregated_inc, and the bucket's box of in-plane key coordinates
// (u, v) (half voxels): the lanes of a group combine their coordinates with
// LDS atomics in a slot of their leader, which then widens the global box
// where it has to.  slot: this wave's 64 x 4 ints of LDS.
__device__ inline void wave_aggregated_inc_box(unsigned int* counter, int4* bbox, long long b, int cu, int cv,
                                               int* slot) {
  unsigned long long todo = __ballot(1);
  const int lane = threadIdx.x & 63;
  unsigned int group = 0;
  int lead = lane;
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const long long bl = __shfl(b, leader, 64);
    const unsigned long long same = __ballot(b == bl) & todo;
    if (b == bl) lead = leader;
    if (lane == leader) group = (unsigned int)__popcll(same);
    todo &= ~same;
  }
  int* s = slot + 4 * lead;
  if (group) {
    s[0] = INT_MAX;
    s[1] = INT_MIN;
    s[2] = INT_MAX;
    s[3] = INT_MIN;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  atomicMin(&s[0], cu);
  atomicMax(&s[1], cu);
  atomicMin(&s[2], cv);
  atomicMax(&s[3], cv);
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (group) {
    atomicAdd(&counter[b], group);
    // The box only grows, so a bound that an earlier (possibly stale) read
    // already covers needs no atomic: most groups of a plane skip all four.
    int* g = (int*)&bbox[b];
    int cur[4];
    for (int j = 0; j < 4; ++j) cur[j] = __hip_atomic_load(&g[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (s[0] < cur[0]) atomicMin(&g[0], s[0]);
    if (s[1] > cur[1]) atomicMax(&g[1], s[1]);
    if (s[2] < cur[2]) atomicMin(&g[2], s[2]);
    if (s[3] > cur[3]) atomicMax(&g[3], s[3]);
  }
  __builtin_amdgcn_wave_barrier();
}

// Row copies of a brick that the scatter orders by destination in LDS.
constexpr int kScatterList = 3072;

// Exclusive prefix sum of s[0, n) in place (n <= 8 * 256, 8 consecutive
// slots per thread of a 256-thread workgroup); returns the sum.  s_w: 4 ints.
// The caller's barrier must precede it; it ends with one.
__device__ inline int block_scan_slots(int* s, int n, int* s_w) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int b = 8 * tid;
  int e[8], sum = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    e[j] = sum;
    sum += b + j < n ? s[b + j] : 0;
  }
  int inc = sum;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(inc, d, 64);
    if (lane >= d) inc += t;
  }
  if (lane == 63) s_w[wid] = inc;
  __syncthreads();
  int base = inc - sum;
  for (int w = 0; w < wid; ++w) base += s_w[w];
  const int total = s_w[0] + s_w[1] + s_w[2] + s_w[3];
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (b + j < n) s[b + j] = base + e[j];
  __syncthreads();
  return total;
}

// A brick's vertices: its rows of layout 0 (consecutive, in the mesh pass's
// order) and its ROI.  False for a brick with no vertex, past the last ROI, or
// of an emptied ROI.
struct BrickRows {
  long long row0, n;
  int roi;
};

__device__ inline bool brick_rows(const BrickArgs& A, long long brick, BrickRows& out) {
  if (brick >= A.nbricks) return false;
  const int r = A.bmap ? A.bmap[brick] : find_roi(A.rois, A.n_rois, brick);
  if (r < 0 || brick >= A.rois[r].brick_end) return false;
  const RoiMeta& M = A.meta[r];
  const long long cnt = A.part[brick].nv, first = A.brick_voff[brick];
  if (cnt == 0 || M.V == 0 || first + cnt > M.V) return false;
  out.row0 = M.row_off + first;
  out.n = cnt;
  out.roi = r;
  return true;
}

// Plane keys of a vertex: along axis j, 2 u_j + [a == j] for the edge
// (u, u + e_a), as bucket indices key + 1 within the ROI's 2 d_j + 1 buckets of
// axis j (a key outside them, which only a stale row could hold, gives -1).
__device__ inline void vertex_buckets(unsigned long long k, const int* d, int* bi, int* kc) {
  const int p[3] = {(int)((k >> 40) & 0xFFFFF), (int)((k >> 20) & 0xFFFFF), (int)(k & 0xFFFFF)};  // u + 1
  const int a = (int)((k >> 60) & 3);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    kc[j] = 2 * (p[j] - 1) + (a == j);
    bi[j] = kc[j] + 1;
    if (bi[j] < 0 || bi[j] > 2 * d[j]) bi[j] = -1;
  }
}

// Calls f(i, key) for every vertex i of the brick; each thread loads the keys
// of four of its rows together, so that their latencies overlap.
template <typename F>
__device__ inline void for_brick_keys(const unsigned long long* __restrict__ key, const BrickRows& W, F&& f) {
  for (long long i4 = threadIdx.x; i4 < W.n; i4 += 4ll * blockDim.x) {
    unsigned long long k[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long long i = i4 + (long long)u * blockDim.x;
      k[u] = i < W.n ? key[W.row0 + i] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long long i = i4 + (long long)u * blockDim.x;
      if (i < W.n) f(i, k[u]);
    }
  }
}

// The brick's window of bucket indices [lo_j, hi_j] per axis (LDS s_lo,
// s_hi); returns the windows' total width (the caller compares it with the
// size of its LDS tables).  Contains barriers.
__device__ inline int brick_windows(const unsigned long long* __restrict__ key, const BrickRows& W, const int* d,
                                    int* s_lo, int* s_hi, int* off) {
  const int tid = threadIdx.x;
  if (tid < 3) {
    s_lo[tid] = INT_MAX;
    s_hi[tid] = INT_MIN;
  }
  __syncthreads();
  int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
  for_brick_keys(key, W, [&](long long, unsigned long long k) {
    int bi[3], kc[3];
    vertex_buckets(k, d, bi, kc);
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (bi[j] >= 0) {
        lo[j] = min(lo[j], bi[j]);
        hi[j] = max(hi[j], bi[j]);
      }
  });
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    lo[j] = wave_min(lo[j]);
    hi[j] = wave_max(hi[j]);
  }
  if ((tid & 63) == 0)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      atomicMin(&s_lo[j], lo[j]);
      atomicMax(&s_hi[j], hi[j]);
    }
  __syncthreads();
  int total = 0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    off[j] = total;
    total += s_hi[j] >= s_lo[j] ? s_hi[j] - s_lo[j] + 1 : 0;
  }
  return total;
}

// Bucket counts, and with bbox set the buckets' boxes in key coordinates (the
// box of a bucket of axis k holds the two other axes in increasing order).
// One workgroup per brick: a brick's vertices lie on few planes of each axis,
// so they are counted per plane in LDS windows and each plane the brick
// touches costs one global atomic (plus the box's, where it grows).  A brick
// whose windows exceed `win` planes uses wave-aggregated global atomics
// per vertex instead.
__global__ __launch_bounds__(256) void k_brick_hist(BrickArgs A, const unsigned long long* __restrict__ key,
                                                    unsigned int* __restrict__ bcnt, int4* __restrict__ bbox, int win) {
  extern __shared__ int s_win[];  // win counts, then with bbox win boxes
  __shared__ int s_lo[3], s_hi[3];
  __shared__ int s_slot[4][64 * 4];
  BrickRows W;
  if (!brick_rows(A, blockIdx.x, W)) return;
  const Roi& R = A.rois[W.roi];
  const int tid = threadIdx.x;
  int off[3];
  const int total = brick_windows(key, W, R.d, s_lo, s_hi, off);
  int* s_box = s_win + win;
  if (total <= win) {
    for (int w = tid; w < total; w += blockDim.x) {
      s_win[w] = 0;
      if (bbox) {
        s_box[4 * w] = INT_MAX;
        s_box[4 * w + 1] = INT_MIN;
        s_box[4 * w + 2] = INT_MAX;
        s_box[4 * w + 3] = INT_MIN;
      }
    }
    __syncthreads();
    // Each thread takes four consecutive vertices at a time and merges runs of
    // equal buckets before its LDS atomics: a brick lists its vertices by
    // row-group, then plane, so their axis-0 and axis-1 buckets repeat, and
    // the same-address atomics of a wave's lanes are serialised.  The box only
    // grows: an atomic that a (possibly stale) read shows cannot change it is
    // skipped.
    auto flush = [&](int w, int c, const int* bx) {
      if (w < 0) return;
      atomicAdd(&s_win[w], c);
      if (bbox) {
        int* q = s_box + 4 * w;
        if (bx[0] < q[0]) atomicMin(&q[0], bx[0]);
        if (bx[1] > q[1]) atomicMax(&q[1], bx[1]);
        if (bx[2] < q[2]) atomicMin(&q[2], bx[2]);
        if (bx[3] > q[3]) atomicMax(&q[3], bx[3]);
      }
    };
    for (long long b0 = 4ll * tid; b0 < W.n; b0 += 4ll * blockDim.x) {
      unsigned long long k[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) k[u] = b0 + u < W.n ? key[W.row0 + b0 + u] : 0ull;
      int cw[3] = {-1, -1, -1}, cc[3] = {0, 0, 0}, bx[3][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (b0 + u >= W.n) continue;
        int bi[3], kc[3];
        vertex_buckets(k[u], R.d, bi, kc);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          if (bi[j] < 0) continue;
          const int w = off[j] + bi[j] - s_lo[j];
          const int cu = kc[j == 0 ? 1 : 0], cv = kc[j == 2 ? 1 : 2];
          if (w != cw[j]) {
            flush(cw[j], cc[j], bx[j]);
            cw[j] = w;
            cc[j] = 0;
            bx[j][0] = bx[j][1] = cu;
            bx[j][2] = bx[j][3] = cv;
          }
          ++cc[j];
          bx[j][0] = min(bx[j][0], cu);
          bx[j][1] = max(bx[j][1], cu);
          bx[j][2] = min(bx[j][2], cv);
          bx[j][3] = max(bx[j][3], cv);
        }
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) flush(cw[j], cc[j], bx[j]);
    }
    __syncthreads();
    for (int w = tid; w < total; w += blockDim.x) {
      const int c = s_win[w];
      if (!c) continue;
      const int j = w >= off[2] ? 2 : (w >= off[1] ? 1 : 0);
      const long long b = R.bucket_base[j] + s_lo[j] + (w - off[j]);
      atomicAdd(&bcnt[b], (unsigned int)c);
      if (bbox) {
        // no read of the global box first: the atomics' results are not
        // waited for, so the workgroup ends without a round trip
        int* g = (int*)&bbox[b];
        const int* q = s_box + 4 * w;
        atomicMin(&g[0], q[0]);
        atomicMax(&g[1], q[1]);
        atomicMin(&g[2], q[2]);
        atomicMax(&g[3], q[3]);
      }
    }
  } else {
    for (long long i = tid; i < W.n; i += blockDim.x) {
      int bi[3], kc[3];
      vertex_buckets(key[W.row0 + i], R.d, bi, kc);
      for (int j = 0; j < 3; ++j) {
        if (bi[j] < 0) continue;  // lanes with an invalid key sit out of the grouping
        const long long b = R.bucket_base[j] + bi[j];
        if (bbox)
          wave_aggregated_inc_box(bcnt, bbox, b, kc[j == 0 ? 1 : 0], kc[j == 2 ? 1 : 2], s_slot[tid >> 6]);
        else
          wave_aggregated_inc(bcnt, b);
      }
    }
  }
}

// Whole plane buckets that cannot hold their family's planar diameter are
// dropped before they are laid out (one workgroup per ROI).  For a family
// (an axis k of a ROI) the two vertices of a bucket with the smallest and the
// largest coordinate along an in-plane axis are a pair of the family, so the
// largest such extent of any bucket, L, bounds the diameter from below; a
// bucket whose box diagonal U satisfies U^2 < L^2 (1 - 2^-20) holds no pair
// that reaches it.  Binary masks: positions are exactly the key coordinates
// times half the spacing.  Soft masks: a vertex lies within half a voxel of
// its key coordinate along its edge's axis, so L uses each extent less one
// voxel, U each extent plus one voxel and, in a bucket of edges along k, one
// voxel along k.  A dropped bucket's count is set to 0 (its in-plane pairs
// still enter the pair statistics).
__global__ __launch_bounds__(256) void k_bucket_prune(const Roi* __restrict__ rois, int soft,
                                                      unsigned int* __restrict__ bcnt, const int4* __restrict__ bbox,
                                                      long long* __restrict__ pairs2d) {
  __shared__ double s_red[4];
  const int r = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const Roi& R = rois[r];
  const double w = soft ? 1.0 : 0.0;
  long long dropped_pairs = 0;
  for (int ax = 0; ax < 3; ++ax) {
    const int ju = ax == 0 ? 1 : 0, jv = ax == 2 ? 1 : 2;
    const double su = R.s[ju], sv = R.s[jv], sk = R.s[ax];
    const long long b0 = R.bucket_base[ax], nb = 2ll * R.d[ax] + 1;
    double L2 = 0.0;
    for (long long i = tid; i < nb; i += 256) {
      if (bcnt[b0 + i] < 2u) continue;
      const int4 q = bbox[b0 + i];
      const double eu = fmax(0.0, 0.5 * (double)(q.y - q.x) - w) * su;
      const double ev = fmax(0.0, 0.5 * (double)(q.w - q.z) - w) * sv;
      L2 = fmax(L2, fmax(eu * eu, ev * ev));
    }
    for (int m = 32; m >= 1; m >>= 1) L2 = fmax(L2, __shfl_xor(L2, m, 64));
    if (lane == 0) s_red[wid] = L2;
    __syncthreads();
    L2 = fmax(fmax(s_red[0], s_red[1]), fmax(s_red[2], s_red[3]));
    __syncthreads();
    const double thr = L2 * (1.0 - 9.5367431640625e-07);  // 1 - 2^-20
    for (long long i = tid; i < nb; i += 256) {
      const unsigned int c = bcnt[b0 + i];
      if (c < 2u) continue;
      const int4 q = bbox[b0 + i];
      const double uu = (0.5 * (double)(q.y - q.x) + w) * su;
      const double vv = (0.5 * (double)(q.w - q.z) + w) * sv;
      const double kk = (soft && (i & 1) == 0) ? sk : 0.0;  // bucket index i = key + 1: odd key <=> even i
      if (uu * uu + vv * vv + kk * kk < thr) {
        bcnt[b0 + i] = 0u;
        dropped_pairs += (long long)c * (c - 1) / 2;
      }
    }
  }
  dropped_pairs = wave_sum(dropped_pairs);
  if (lane == 0 && dropped_pairs) atomicAdd((unsigned long long*)&pairs2d[r], (unsigned long long)dropped_pairs);
}

// Clears the bucket counters, boxes (if any) and the per-ROI in-plane pair
// counts (one launch).
__global__ void k_zero_buckets(unsigned int* __restrict__ bcnt, unsigned int* __restrict__ bcur, long long nb,
                               long long* __restrict__ pairs2d, long long n_rois, int4* __restrict__ bbox) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += stride) {
    bcnt[i] = 0u;
    bcur[i] = 0u;
    if (bbox) bbox[i] = make_int4(INT_MAX, INT_MIN, INT_MAX, INT_MIN);
  }
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_rois; i += stride) pairs2d[i] = 0;
}

__global__ void k_bucket_sizes(const unsigned int* __restrict__ bcnt, long long nb, long long* __restrict__ bsz,
                               long long* __restrict__ bflag) {
  for (long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += (long long)gridDim.x * blockDim.x) {
    const unsigned int c = bcnt[b];
    bsz[b] = c >= 2 ? (long long)((c + kSegAlign - 1) / kSegAlign * kSegAlign) : 0;
    bflag[b] = c >= 2 ? 1 : 0;
  }
}

// Copies every vertex's operand row into its three plane buckets (those with
// at least two vertices after pruning), at rows0 + brow[b] + slot.  One
// workgroup per brick: the brick counts its vertices per plane in LDS, takes
// its slots of each plane with one global atomic, and orders its copies by
// destination in LDS (a counting sort) before writing them.  A brick whose
// windows exceed `win` planes groups the lanes of
// a wave per bucket and issues one global atomic per group instead.
__global__ __launch_bounds__(256) void k_brick_scatter(BrickArgs A, const unsigned long long* __restrict__ key,
                                                       const long long* __restrict__ totals,
                                                       const unsigned int* __restrict__ bcnt,
                                                       unsigned int* __restrict__ bcur,
                                                       const long long* __restrict__ brow, float* __restrict__ pos,
                                                       uint4* __restrict__ posh, int* __restrict__ orig, int win) {
  extern __shared__ int s_win[];  // win counts, then win offsets, then kScatterList entries
  __shared__ int s_lo[3], s_hi[3], s_sw[4];
  BrickRows W;
  if (!brick_rows(A, blockIdx.x, W)) return;
  const Roi& R = A.rois[W.roi];
  const long long rows0 = totals[T_ROWS0];
  const int tid = threadIdx.x, lane = tid & 63;
  int off[3];
  const int total = brick_windows(key, W, R.d, s_lo, s_hi, off);
  if (total <= win) {
    int* s_rel = s_win + win;
    unsigned int* s_list = (unsigned int*)(s_win + 2 * win);
    for (int w = tid; w < total; w += blockDim.x) s_win[w] = 0;
    __syncthreads();
    for_brick_keys(key, W, [&](long long, unsigned long long k) {
      int bi[3], kc[3];
      vertex_buckets(k, R.d, bi, kc);
#pragma unroll
      for (int j = 0; j < 3; ++j)
        if (bi[j] >= 0) atomicAdd(&s_win[off[j] + bi[j] - s_lo[j]], 1);
    });
    __syncthreads();
    // the brick's slots in each plane bucket (kept ones only): rows brow[b] + base ...
    for (int w = tid; w < total; w += blockDim.x) {
      const int c = s_win[w];
      int rel = INT_MIN;
      if (c) {
        const int j = w >= off[2] ? 2 : (w >= off[1] ? 1 : 0);
        const long long b = R.bucket_base[j] + s_lo[j] + (w - off[j]);
        if (bcnt[b] >= 2u) rel = (int)(brow[b] + (long long)atomicAdd(&bcur[b], (unsigned int)c));
      }
      s_rel[w] = rel;
      s_win[w] = rel == INT_MIN ? 0 : c;
    }
    __syncthreads();
    // ... and the brick's copies listed by destination: window w's copies take
    // list positions [pre_w, pre_w + c_w), and position q goes to row
    // rows0 + brow[b] + base + (q - pre_w) = rows0 + s_rel[w] + q
    const int n_copy = block_scan_slots(s_win, total, s_sw);
    for (int w = tid; w < total; w += blockDim.x)
      if (s_rel[w] != INT_MIN) s_rel[w] -= s_win[w];
    __syncthreads();
    // Listed, the copies are written in destination order, so neighbouring
    // lanes fill neighbouring rows (whole cache lines) instead of one row of
    // a different bucket each; a brick with more copies than the list holds
    // writes them directly.
    const bool listed = n_copy <= kScatterList && W.n < (1ll << 21);
    for_brick_keys(key, W, [&](long long i, unsigned long long k) {
      int bi[3], kc[3];
      vertex_buckets(k, R.d, bi, kc);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        if (bi[j] < 0) continue;
        const int w = off[j] + bi[j] - s_lo[j];
        if (s_rel[w] == INT_MIN) continue;
        const int q = atomicAdd(&s_win[w], 1);
        if (listed) {
          s_list[q] = ((unsigned int)w << 21) | (unsigned int)i;
        } else {
          const long long row = W.row0 + i, dst_row = rows0 + s_rel[w] + q;
          copy_row_operands(pos, posh, row, dst_row);
          orig[dst_row] = (int)row;
        }
      }
    });
    if (listed) {
      __syncthreads();
      for (int q = tid; q < n_copy; q += blockDim.x) {
        const unsigned int e = s_list[q];
        const long long row = W.row0 + (e & 0x1fffffu), dst_row = rows0 + s_rel[e >> 21] + q;
        copy_row_operands(pos, posh, row, dst_row);
        orig[dst_row] = (int)row;
      }
    }
  } else {
    for (long long i0 = 0; i0 < W.n; i0 += blockDim.x) {
      const long long i = i0 + tid;
      const long long row = W.row0 + i;
      long long b[3] = {0, 0, 0};
      bool on[3] = {false, false, false};
      if (i < W.n) {
        int bi[3], kc[3];
        vertex_buckets(key[row], R.d, bi, kc);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          b[j] = R.bucket_base[j] + bi[j];
          on[j] = bi[j] >= 0 && bcnt[b[j]] >= 2u;
        }
      }
      // the three buckets' slots: lanes are grouped per axis by bucket (ALU
      // only) and the leaders' atomics are all issued before any result is used
      unsigned int base[3] = {0u, 0u, 0u}, rank[3] = {0u, 0u, 0u};
      int lead[3] = {lane, lane, lane};
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        unsigned long long todo = __ballot(on[j]);
        unsigned int group = 0;
        while (todo) {
          const int leader = __ffsll((long long)todo) - 1;
          const long long bl = __shfl(b[j], leader, 64);
          const bool mine = on[j] && b[j] == bl;
          const unsigned long long same = __ballot(mine) & todo;
          if (mine) {
            lead[j] = leader;
            rank[j] = (unsigned int)__popcll(same & ((1ull << lane) - 1ull));
          }
          if (lane == leader) group = (unsigned int)__popcll(same);
          todo &= ~same;
        }
        if (group) base[j] = atomicAdd(&bcur[b[j]], group);
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const unsigned int slot = __shfl(base[j], lead[j], 64) + rank[j];
        if (!on[j]) continue;
        const long long dst_row = rows0 + brow[b[j]] + slot;
        copy_row_operands(pos, posh, row, dst_row);
        orig[dst_row] = (int)row;
      }
    }
  }
}

// The group (roi * 4 + 1 + axis) of every plane bucket, and the ROI's
// in-plane pair count n (n - 1) / 2 summed over its kept buckets (one atomic
// per ROI: the pruning pass adds the dropped buckets' pairs): one workgroup
// per ROI over its contiguous bucket range (so the segment pass needs no
// search of the ROI table).
__global__ __launch_bounds__(256) void k_bucket_groups(const Roi* __restrict__ rois, int* __restrict__ bgroup,
                                                       const unsigned int* __restrict__ bcnt,
                                                       long long* __restrict__ pairs2d) {
  __shared__ long long s_sum[4];
  const Roi& R = rois[blockIdx.x];
  const long long b0 = R.bucket_base[0];
  const long long b1 = R.bucket_base[2] + 2ll * R.d[2] + 1;
  long long pairs = 0;
  for (long long b = b0 + threadIdx.x; b < b1; b += blockDim.x) {
    const int axis = b >= R.bucket_base[2] ? 2 : (b >= R.bucket_base[1] ? 1 : 0);
    bgroup[b] = (int)blockIdx.x * 4 + 1 + axis;
    const long long c = bcnt[b];
    if (c >= 2) pairs += c * (c - 1) / 2;
  }
  pairs = wave_sum(pairs);
  if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = pairs;
  __syncthreads();
  if (threadIdx.x == 0) {
    const long long t = s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3];
    if (t) atomicAdd((unsigned long long*)&pairs2d[blockIdx.x], (unsigned long long)t);
  }
}

// Segments of the buckets: pad rows, block tags and the segment table.
__global__ void k_bucket_segs(const int* __restrict__ bgroup, int n_rois, long long nb,
                              const long long* __restrict__ totals,
                              const unsigned int* __restrict__ bcnt, const long long* __restrict__ bsz,
                              const long long* __restrict__ brow, const long long* __restrict__ bseg,
                              float* __restrict__ pos, uint4* __restrict__ posh, int* __restrict__ orig,
                              int* __restrict__ blkseg, Seg* __restrict__ segs, int per_wave) {
  // A wave takes per_wave buckets at a time (64 in calls with many buckets,
  // most of them empty or pruned; else 1), a lane each, and loads their counts
  // and offsets together; then the whole wave serves each bucket of two or
  // more vertices in turn: its lanes tag the blocks and fill the pad rows.
  const long long rows0 = totals[T_ROWS0];
  const int lane = threadIdx.x & 63;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long b0 = (((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * per_wave; b0 < nb;
       b0 += nwaves * per_wave) {
    const long long bl = b0 + lane;
    const unsigned int cl = lane < per_wave && bl < nb ? bcnt[bl] : 0u;
    long long sidl = 0, r0l = 0, nl = 0;
    int groupl = 0, ol = 0;
    if (cl >= 2u) {
      sidl = n_rois + bseg[bl];
      r0l = rows0 + brow[bl];
      nl = bsz[bl];
      groupl = bgroup[bl];
      ol = orig[r0l];
    }
    unsigned long long todo = __ballot(cl >= 2u);
    while (todo) {
      const int src = __ffsll((long long)todo) - 1;
      todo &= todo - 1ull;
      const unsigned int c = (unsigned int)__shfl((int)cl, src, 64);
      const long long sid = __shfl(sidl, src, 64), r0 = __shfl(r0l, src, 64), n = __shfl(nl, src, 64);
      const int group = __shfl(groupl, src, 64), o = __shfl(ol, src, 64);
      if (lane == 0) {
        Seg S;
        S.row_begin = r0;
        S.n_rows = (int)n;
        S.group = group;
        segs[sid] = S;
      }
      for (long long i = lane; i < n / kBlk; i += 64) blkseg[r0 / kBlk + i] = (int)sid;
      for (long long row = r0 + c + lane; row < r0 + n; row += 64) {
        copy_row_operands(pos, posh, r0, row);
        orig[row] = o;
      }
    }
  }
}

// Columns (chunks of jchunk row blocks) per segment; also clears the item
// counts of all col_cap columns (k_col_fill sets those of the real ones).
// With prune set, the pruned ROIs' 3D segments are left out (the pruned item
// list covers them) unless that list overflowed (counters[4]).
__global__ void k_seg_cols(int n_rois, long long seg_cap, const long long* __restrict__ totals,
                           const Seg* __restrict__ segs, const RoiMeta* __restrict__ meta,
                           long long* __restrict__ ncol, int jchunk, int small_rows,
                           long long* __restrict__ nitem, long long col_cap, int prune, int prune_min_v,
                           const unsigned int* __restrict__ counters) {
  const long long nseg = n_rois + totals[T_NSEG2D];
  const bool skip3d = prune && counters[4] == 0u;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < col_cap;
       c += (long long)gridDim.x * blockDim.x)
    nitem[c] = 0;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < seg_cap;
       s += (long long)gridDim.x * blockDim.x) {
    long long rows = s < nseg ? segs[s].n_rows : 0;
    if (s >= n_rois && rows <= small_rows) rows = 0;  // a small bucket: k_pair_small_h
    if (s < n_rois && skip3d && meta[s].V >= prune_min_v) rows = 0;  // a pruned 3D segment: k_pair_list_h
    ncol[s] = (rows + (long long)jchunk * kBlk - 1) / ((long long)jchunk * kBlk);
  }
}

// Column table and items per column: items of column jc of a segment are the
// row tiles (itile blocks) that start before the column ends (upper triangle).
__global__ void k_col_fill(int n_rois, long long seg_cap, const long long* __restrict__ totals,
                           const Seg* __restrict__ segs, const RoiMeta* __restrict__ meta,
                           const long long* __restrict__ ncol,
                           const long long* __restrict__ colbase, Col* __restrict__ cols,
                           long long* __restrict__ nitem, int itile, int jchunk) {
  const long long nseg = n_rois + totals[T_NSEG2D];
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < nseg; s += (long long)gridDim.x * blockDim.x) {
    const long long nc = ncol[s];
    if (nc == 0) continue;
    const Seg S = segs[s];
    const long long nblk = S.n_rows / kBlk;
    const long long nt = (nblk + itile - 1) / itile;
    const int e = h_scale_exp(meta[S.group >> 2].R2);
    for (long long jc = 0; jc < nc; ++jc) {
      const long long c = colbase[s] + jc;
      Col C;
      C.row_begin = S.row_begin;
      C.n_rows = S.n_rows;
      C.group = S.group;
      C.jc = (int)jc;
      C.e = e;
      cols[c] = C;
      const long long lim = (jc + 1) * (jchunk / itile);
      nitem[c] = nt < lim ? nt : lim;
    }
  }
}

// ---------------------------------------------------------------------------
// Pair maxima on the matrix cores.

// Hands the work items [0, n) out to waves.  The items are split into
// kWorkParts contiguous ranges, each with its own counter (kWorkStride words
// apart, so the counters sit in different cache lines and their atomics do not
// queue behind one another; one shared counter serialises its atomics at
// roughly one per 18 ns, which bounded batches of small ROIs with millions of
// items).  A wave starts on the range of its workgroup's XCD (workgroups are
// dispatched round-robin over the 8 XCDs), takes `grab` consecutive items per
// atomic (two when there are at least 8 items per wave, else one), and moves on
// to the following ranges once its range is exhausted.  A range it moves on to
// is first read with a plain device-scope load, so that the usual case at the
// end (every range already exhausted) costs loads, which do not queue, rather
// than atomics.  Every wave ends after at most kWorkParts failed grabs.  All
// members are wave-uniform.  (Reading all counters at once with a ballot was
// tried: the kernel then needs more than 168 VGPRs and loses a wave per SIMD.)
struct WorkQueue {
  unsigned int* ctr;
  long long n, cur, end, lo, hi;
  int part, left, grab;
  bool look;  // read the current range's counter before the next atomic

  __device__ WorkQueue(unsigned int* c, long long n_items)
      : ctr(c), n(n_items), cur(0), end(0), part((int)(blockIdx.x % kWorkParts)), left(kWorkParts), look(false) {
    const long long waves = (long long)gridDim.x * (blockDim.x >> 6);
    grab = n_items >= 8 * waves ? 2 : 1;
    set_range();
  }
  __device__ void set_range() {
    lo = n * part / kWorkParts;
    hi = n * (part + 1) / kWorkParts;
  }
  // The next item, or -1 once every range is exhausted.
  __device__ long long next(int lane) {
    if (cur < end) return cur++;
    while (left > 0) {
      unsigned int got = 0;
      if (lane == 0) {
        unsigned int* c = ctr + part * kWorkStride;
        if (look) got = __hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!look || lo + (long long)got * grab < hi) got = atomicAdd(c, 1u);
      }
      const long long first = lo + (long long)__builtin_amdgcn_readfirstlane((int)__shfl(got, 0, 64)) * grab;
      if (first < hi) {
        cur = first + 1;
        end = min(first + grab, hi);
        look = false;
        return first;
      }
      --left;
      part = (part + 1) % kWorkParts;
      set_range();
      look = true;
    }
    return -1;
  }
};

// The column of an item: the last column whose first item is <= item (empty
// columns share their base with the next one).  A wave's items mostly ascend
// within a range, so the cached column is walked forward a few steps before
// falling back to a binary search.
struct ColumnOf {
  const long long* itembase;
  long long n_items, ncol, col, col_lo, col_hi;

  __device__ ColumnOf(const long long* ib, long long ni, long long nc)
      : itembase(ib), n_items(ni), ncol(nc), col(0), col_lo(0), col_hi(nc > 1 ? ib[1] : ni) {}
  __device__ void advance() {
    ++col;
    col_lo = col_hi;
    col_hi = col + 1 < ncol ? itembase[col + 1] : n_items;
  }
  __device__ void locate(long long item) {
    for (int steps = 0; steps < 4 && item >= col_hi; ++steps) advance();
    if (item < col_lo || item >= col_hi) {
      long long lo2 = item < col_lo ? 0 : col, hi2 = ncol - 1;
      while (lo2 < hi2) {
        const long long mid = (lo2 + hi2 + 1) >> 1;
        if (itembase[mid] <= item)
          lo2 = mid;
        else
          hi2 = mid - 1;
      }
      col = lo2;
      col_lo = itembase[col];
      col_hi = col + 1 < ncol ? itembase[col + 1] : n_items;
    }
    while (col + 1 < ncol && item >= col_hi) advance();
  }
};

// 2*IT MFMAs: the IT row blocks against two column blocks, folded into the
// running row maxima with v_max3.
template <int IT>
__device__ __forceinline__ void pair_tile(const float (&A)[IT], float b0, float b1, v4f (&acc)[IT]) {
  const v4f zero = {0.f, 0.f, 0.f, 0.f};
  v4f d[2 * IT];
#pragma unroll
  for (int r = 0; r < IT; ++r) {
    d[2 * r] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[r], b0, zero, 0, 0, 0);
    d[2 * r + 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[r], b1, zero, 0, 0, 0);
  }
  // One v_max3 per two pair values (the floor: the matrix core and the VALU do
  // not co-execute, so every VALU cycle adds to the MFMA cycles).  The empty asm
  // pins the running maximum after each tile so the compiler cannot
  // re-associate two tiles into max/max/max3 (three ops per four values).
#pragma unroll
  for (int r = 0; r < IT; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float a = fmaxf(acc[r][q], fmaxf(d[2 * r][q], d[2 * r + 1][q]));
      asm volatile("" : "+v"(a));
      acc[r][q] = a;
    }
}

template <int IT>
__global__ __launch_bounds__(256) void k_pair_maxima(const float* __restrict__ pos, const Col* __restrict__ cols,
                                                     const long long* __restrict__ itembase,
                                                     const long long* __restrict__ totals,
                                                     unsigned int* __restrict__ work_ctr, float* __restrict__ rowmax,
                                                     int jchunk) {
  const int lane = threadIdx.x & 63;
  WorkQueue q(work_ctr, totals[T_NITEM]);
  ColumnOf where(itembase, totals[T_NITEM], totals[T_NCOL]);
  for (long long item; (item = q.next(lane)) >= 0;) {
    where.locate(item);
    const Col C = cols[where.col];
    const int it = (int)(item - where.col_lo);
    const long long rb = C.row_begin >> 4;
    const int nb = C.n_rows >> 4;
    const int i0 = it * IT;
    const int j0 = max(C.jc * jchunk, i0);
    const int j1 = min((C.jc + 1) * jchunk, nb);

    float A[IT];
#pragma unroll
    for (int r = 0; r < IT; ++r) {
      const int blk = min(i0 + r, nb - 1);
      const float v = pos[(rb + blk) * 64 + lane];
      A[r] = lane < 48 ? -2.0f * v : 1.0f;
    }
    v4f acc[IT];
#pragma unroll
    for (int r = 0; r < IT; ++r) acc[r] = v4f{-3.0e38f, -3.0e38f, -3.0e38f, -3.0e38f};

    // Column blocks are consumed in pairs; two pairs are kept in flight
    // (double buffering).  Prefetch addresses are clamped to the last pair of
    // the range so every load stays inside the segment, and a clamped pair is
    // simply processed twice.
    const float* B = pos + rb * 64 + lane;
    float b0 = B[j0 * 64], b1 = B[(j0 + 1) * 64];
    for (int jb = j0; jb < j1; jb += 4) {
      const int jn = min(jb + 2, j1 - 2);
      const float c0 = B[jn * 64], c1 = B[(jn + 1) * 64];
      pair_tile(A, b0, b1, acc);
      const int jm = min(jb + 4, j1 - 2);
      b0 = B[jm * 64];
      b1 = B[(jm + 1) * 64];
      pair_tile(A, c0, c1, acc);  // repeats the last pair when the pair count is odd: harmless for a max
    }
    // D[i][j] sits in lane 16*(i/4) + j, register i%4: reduce over j (the low 4 lane bits)
#pragma unroll
    for (int r = 0; r < IT; ++r) {
      if (i0 + r >= nb) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float m = acc[r][q];
        m = fmaxf(m, __shfl_xor(m, 1, 64));
        m = fmaxf(m, __shfl_xor(m, 2, 64));
        m = fmaxf(m, __shfl_xor(m, 4, 64));
        m = fmaxf(m, __shfl_xor(m, 8, 64));
        if ((lane & 15) == q) {
          const long long row = (rb + i0 + r) * 16 + 4 * (lane >> 4) + q;
          const float w = pos[(rb + i0 + r) * 64 + 48 + 4 * (lane >> 4) + q];
          const float val = fmaxf(m + w, 0.0f);
          atomicMax((int*)&rowmax[row], __float_as_int(val));
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Split-f16 pair maxima on the 32x32x16 f16 matrix cores.
//
// Each centred FP32 coordinate, scaled by 2^e (h_scale_exp), is split into
// h = f16(x) and l = f16(x - h); x_i . x_j is then h_i.h_j + h_i.l_j + l_i.h_j
// up to l_i.l_j ~ 2^-22 |x_i||x_j|, and w = |x|^2 likewise splits into two
// f16.  One K = 16 contraction gives the whole squared distance:
//   A_i = [-2h, -2h, -2l, w_hi, w_lo, 1, 1, 0, 0, 0]_i   (3+3+3+1+1+1+1+3)
//   B_j = [ h,   l,   h,  1,    1,  w_hi, w_lo, 0, 0, 0]_j
// so a v_mfma_f32_32x32x16_f16 yields 1024 pair values (FP32 accumulation)
// for the cost of a quarter of the FP32 16x16x4 instructions per pair.  The
// bound on the error (a few 2^-18 R^2, see k_candidates) is covered by the
// exact FP64 refinement that follows.
//
// Operand layout (posh): 32 B per row, the B operand's K entries 0-7 then
// 8-15 (write_split_row); lane l of a wave takes K entries 8*(l/32) ..
// 8*(l/32)+7 of row l % 32, so a 32-row block is one contiguous 1 KB load.
// The A operand, needed once per work item, is rebuilt from B in registers
// (a_from_b).

typedef float v16f __attribute__((ext_vector_type(16)));

// The A operand of a 32-row block from its B operand, in registers: lanes
// 0-31 (K 0-7) get -2 [h, h, l0, l1] from their own B entries, lanes 32-63
// (K 8-15) get [-2 l2, w_hi, w_lo, 1, 1, 0, 0, 0], with l2 taken from the
// partner lane (lane ^ 32).  Scaling by -2 is exact in f16.
__device__ __forceinline__ v8h a_from_b(const uint4& u, int lane) {
  const v8h b = *(const v8h*)&u;
  const unsigned int pz = __shfl_xor(u.z, 32, 64);  // entries 4, 5 of the partner lane's B
  const _Float16 l2 = __builtin_bit_cast(_Float16, (unsigned short)(pz >> 16));
  const _Float16 m2 = (_Float16)-2.0f, one = (_Float16)1.0f, zero = (_Float16)0.0f;
  const v8h lo = {m2 * b[0], m2 * b[1], m2 * b[2], m2 * b[0], m2 * b[1], m2 * b[2], m2 * b[3], m2 * b[4]};
  const v8h hi = {m2 * l2, b[3], b[4], one, one, zero, zero, zero};
  return lane < 32 ? lo : hi;
}

// 2*IT MFMAs: the IT row blocks against two column blocks, folded into the
// running maxima with v_max3 (one per two pair values, as in pair_tile).
template <int IT>
__device__ __forceinline__ void pair_tile_h(const v8h (&A)[IT], const v8h& b0, const v8h& b1, v16f (&acc)[IT]) {
  const v16f zero = {};
#pragma unroll
  for (int r = 0; r < IT; ++r) {
    const v16f d0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(A[r], b0, zero, 0, 0, 0);
    const v16f d1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(A[r], b1, zero, 0, 0, 0);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      float a = fmaxf(acc[r][q], fmaxf(d0[q], d1[q]));
      asm volatile("" : "+v"(a));
      acc[r][q] = a;
    }
  }
}

// One tile of the split-f16 pair pass: 32-row blocks i0 .. i0 + IT - 1 of the
// segment starting at block rb (nb blocks) against its column blocks
// [j0, j1), folded into the row maxima (scale exponent e of the ROI).
template <int IT>
__device__ __forceinline__ void pair_item_h(const uint4* __restrict__ posh, float* __restrict__ rowmax, long long rb,
                                            int nb, int i0, int j0, int j1, int e, int lane) {
  v8h A[IT];
#pragma unroll
  for (int r = 0; r < IT; ++r) {
    const int blk = min(i0 + r, nb - 1);
    A[r] = a_from_b(posh[(rb + blk) * 64 + split_lane_index(lane)], lane);
  }
  v16f acc[IT];
#pragma unroll
  for (int r = 0; r < IT; ++r)
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[r][q] = -3.0e38f;

  // column blocks in pairs, two pairs in flight; indices clamped to the last
  // block of the range (a repeated block is harmless for a maximum)
  const uint4* Bp = posh + rb * 64 + split_lane_index(lane);
  const int jl = j1 - 1;
  uint4 u0 = Bp[(long long)j0 * 64], u1 = Bp[(long long)min(j0 + 1, jl) * 64];
  for (int jb = j0; jb < j1; jb += 4) {
    const uint4 u2 = Bp[(long long)min(jb + 2, jl) * 64], u3 = Bp[(long long)min(jb + 3, jl) * 64];
    pair_tile_h<IT>(A, *(const v8h*)&u0, *(const v8h*)&u1, acc);
    u0 = Bp[(long long)min(jb + 4, jl) * 64];
    u1 = Bp[(long long)min(jb + 5, jl) * 64];
    pair_tile_h<IT>(A, *(const v8h*)&u2, *(const v8h*)&u3, acc);
  }
  // D[i][j] sits in lane j + 32 * ((i / 4) % 2), register 4 * (i / 8) + i % 4
  // of acc[r]: reduce over j (the low 5 lane bits) with a butterfly that
  // halves the registers at every step (lane bit s keeps one half and sends
  // the other), 62 shuffles for 64 registers.  Afterwards a lane holds the
  // maxima of registers t + 2 * rev5(lane & 31), t = 0, 1, of the flat
  // index r * 16 + q; then undo the scale.
  float v[16 * IT];
#pragma unroll
  for (int r = 0; r < IT; ++r)
#pragma unroll
    for (int q = 0; q < 16; ++q) v[16 * r + q] = acc[r][q];
#pragma unroll
  for (int st = 0; st < 5; ++st) {
    const int h = (16 * IT) >> (st + 1);
    const bool hi = (lane >> st) & 1;
#pragma unroll
    for (int t = 0; t < h; ++t) {
      const float keep = hi ? v[t + h] : v[t], send = hi ? v[t] : v[t + h];
      v[t] = fmaxf(keep, __shfl_xor(send, 1 << st, 64));
    }
  }
  const int rev = ((lane & 1) << 4) | ((lane & 2) << 2) | (lane & 4) | ((lane & 8) >> 2) | ((lane & 16) >> 4);
  const float unscale = ldexpf(1.0f, -2 * e);
#pragma unroll
  for (int t = 0; t < (16 * IT) / 32; ++t) {
    const int flat = t + ((16 * IT) / 32) * rev;  // register index r * 16 + q
    const int r = flat >> 4, q = flat & 15;
    if (i0 + r >= nb) continue;
    const int i = 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
    const long long row = (rb + i0 + r) * 32 + i;
    const float val = fmaxf(v[t], 0.0f) * unscale;
    atomicMax((int*)&rowmax[row], __float_as_int(val));
  }
}

// Work items as for k_pair_maxima with itile = 2 * IT 16-row blocks: IT
// 32-row blocks of A against the column chunk's 32-row blocks of B.
template <int IT>
__global__ __launch_bounds__(256) void k_pair_maxima_h(const uint4* __restrict__ posh, const Col* __restrict__ cols,
                                                       const long long* __restrict__ itembase,
                                                       const long long* __restrict__ totals,
                                                       unsigned int* __restrict__ work_ctr,
                                                       float* __restrict__ rowmax, int jchunk) {
  const int lane = threadIdx.x & 63;
  WorkQueue q(work_ctr, totals[T_NITEM]);
  ColumnOf where(itembase, totals[T_NITEM], totals[T_NCOL]);
  for (long long item; (item = q.next(lane)) >= 0;) {
    where.locate(item);
    const Col C = cols[where.col];  // the segment's rows and scale travel with the column
    const int it = (int)(item - where.col_lo);
    // 32-row block coordinates (segments start and end on 32-row boundaries)
    const long long rb = C.row_begin >> 5;
    const int nb = C.n_rows >> 5;
    const int e = C.e;
    const int i0 = it * IT;
    const int j0 = max(C.jc * (jchunk >> 1), i0);
    const int j1 = min((C.jc + 1) * (jchunk >> 1), nb);
    pair_item_h<IT>(posh, rowmax, rb, nb, i0, j0, j1, e, lane);
  }
}

// The pruned 3D work items (prune.hip): the same tiles as the work-list
// kernel, read from an explicit list of (segment, row tile, column blocks).
// The list is empty when it overflowed (the 3D segments are then in the
// work list).
template <int IT>
__global__ __launch_bounds__(256) void k_pair_list_h(const uint4* __restrict__ posh, const PItem* __restrict__ items,
                                                     const unsigned int* __restrict__ counters, long long cap,
                                                     unsigned int* __restrict__ work_ctr,
                                                     float* __restrict__ rowmax) {
  const int lane = threadIdx.x & 63;
  const long long n = counters[4] != 0u ? 0 : min((long long)counters[3], cap);
  WorkQueue q(work_ctr, n);
  for (long long item; (item = q.next(lane)) >= 0;) {
    const PItem P = items[item];
    pair_item_h<IT>(posh, rowmax, P.rb, P.nb, P.i0, P.j0, P.j1, P.e, lane);
  }
}

// Plane buckets of at most kSmallBlocks 32-row blocks (most of them), which the
// work list leaves out: a wave takes kSmallPerWave consecutive bucket segments
// and runs their row tiles directly, without the work counter and the column
// look-ups, whose chain of dependent loads dominated such small items.
template <int IT>
__global__ __launch_bounds__(256) void k_pair_small_h(const uint4* __restrict__ posh, const Seg* __restrict__ segs,
                                                      int n_rois, const long long* __restrict__ totals,
                                                      const RoiMeta* __restrict__ meta, float* __restrict__ rowmax) {
  const int lane = threadIdx.x & 63;
  const long long nseg2d = totals[T_NSEG2D];
  const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const long long s0 = wave * kSmallPerWave;
  if (s0 >= nseg2d) return;
  Seg S[kSmallPerWave];
#pragma unroll
  for (int k = 0; k < kSmallPerWave; ++k) {
    S[k].n_rows = 0;
    if (s0 + k < nseg2d) S[k] = segs[n_rois + s0 + k];
  }
#pragma unroll
  for (int k = 0; k < kSmallPerWave; ++k) {
    const int nb = S[k].n_rows >> 5;
    if (nb == 0 || nb > kSmallBlocks) continue;
    const int e = h_scale_exp(meta[S[k].group >> 2].R2);
    const long long rb = S[k].row_begin >> 5;
    for (int i0 = 0; i0 < nb; i0 += IT) pair_item_h<IT>(posh, rowmax, rb, nb, i0, i0, nb, e, lane);
  }
}

// ---------------------------------------------------------------------------
// Exact refinement.

// Group maxima of the FP32 row maxima.  Each lane reduces one 16-row block
// (a block lies in one segment, hence one group); each wave then issues one
// atomic per distinct group among its 64 blocks (usually one).
__global__ void k_group_max(const float* __restrict__ rowmax, const int* __restrict__ blkseg,
                            const Seg* __restrict__ segs, const long long* __restrict__ totals,
                            GroupRes* __restrict__ gres) {
  // A wave takes a contiguous range of 16-row blocks, 64 at a time, and keeps
  // the maximum of the group it last met: a group (a ROI's 3D rows, or one
  // axis's plane buckets) covers long runs of blocks, so it costs one atomic
  // per wave that meets it, instead of one per wave and 64 blocks (the
  // atomics of a group serialise on its one address).
  const long long nblk = (totals[T_ROWS0] + totals[T_ROWS2D]) / kBlk;
  const int lane = threadIdx.x & 63;
  const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  const long long per = (nblk + nwaves - 1) / nwaves;
  const long long b0 = wave * per, b1 = min(b0 + per, nblk);
  int cg = -1;  // the group whose maximum cm the wave holds (uniform over the wave)
  float cm = 0.0f;
  for (long long base = b0; base < b1; base += 64) {
    const long long blk = base + lane;
    int g = -1;
    float m = 0.0f;
    if (blk < b1) {
      const int sg = blkseg[blk];
      if (sg >= 0) {
        g = segs[sg].group;
        const float4* p = (const float4*)(rowmax + blk * kBlk);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float4 v = p[i];
          m = fmaxf(m, fmaxf(fmaxf(v.x, v.y), fmaxf(v.z, v.w)));
        }
      }
    }
    unsigned long long todo = __ballot(g >= 0);
    while (todo) {
      const int leader = __ffsll((long long)todo) - 1;
      const int gl = __shfl(g, leader, 64);
      const unsigned long long same = __ballot(g == gl) & todo;
      float v = g == gl ? m : 0.0f;
      for (int k = 32; k >= 1; k >>= 1) v = fmaxf(v, __shfl_xor(v, k, 64));
      if (gl == cg) {
        cm = fmaxf(cm, v);
      } else {
        if (cg >= 0 && lane == 0) atomicMax((int*)&gres[cg].gmax, __float_as_int(cm));
        cg = gl;
        cm = v;
      }
      todo &= ~same;
    }
  }
  if (cg >= 0 && lane == 0) atomicMax((int*)&gres[cg].gmax, __float_as_int(cm));
}

__global__ void k_candidates(const float* __restrict__ rowmax, const int* __restrict__ blkseg,
                             const Seg* __restrict__ segs, const RoiMeta* __restrict__ meta,
                             const long long* __restrict__ totals, GroupRes* __restrict__ gres,
                             unsigned int* __restrict__ ncand, int* __restrict__ cand, long long cand_cap,
                             double band) {
  // A thread per 16-row block (a block lies in one segment: one threshold and
  // one set of look-ups for its 16 rows); a wave reserves its candidates'
  // slots with one atomic.
  const long long nblk = (totals[T_ROWS0] + totals[T_ROWS2D]) / kBlk;
  const int lane = threadIdx.x & 63;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long base = (long long)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < nblk; base += stride) {
    const long long blk = base + lane;
    unsigned int mask = 0u;
    int g = 0;
    const int s = blk < nblk ? blkseg[blk] : -1;
    if (s >= 0) {
      const Seg S = segs[s];
      g = S.group;
      const float gm = S.n_rows > 0 ? gres[g].gmax : 0.0f;
      if (gm > 0.0f) {
        // A pair value of the MFMA pass differs from the exact squared
        // distance by less than half of band * max(R^2, d2) (FP32 Gram form:
        // 2^-18; split f16: 2^-16, see the pass); keep every row within that
        // band of the group maximum.
        const double R2 = meta[g >> 2].R2;
        const float tau = (float)((double)gm - band * (R2 > (double)gm ? R2 : (double)gm));
        const float4* p = (const float4*)(rowmax + blk * kBlk);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float4 v = p[q];
          mask |= ((unsigned int)(v.x >= tau) | ((unsigned int)(v.y >= tau) << 1) |
                   ((unsigned int)(v.z >= tau) << 2) | ((unsigned int)(v.w >= tau) << 3))
                  << (4 * q);
        }
      }
    }
    const int cnt = __popc(mask);
    int inc = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int t = __shfl_up(inc, d, 64);
      if (lane >= d) inc += t;
    }
    const int total = __shfl(inc, 63, 64);
    if (total == 0) continue;
    unsigned int first = 0;
    if (lane == 63) first = atomicAdd(ncand, (unsigned int)total);
    first = __shfl(first, 63, 64);
    unsigned int idx = first + (unsigned int)(inc - cnt);
    while (mask) {
      const int i = __ffs(mask) - 1;
      mask &= mask - 1u;
      if (idx < cand_cap) cand[idx] = (int)(blk * kBlk + i);
      ++idx;
    }
    if (cnt) atomicAdd(&gres[g].n_cand, cnt);
  }
}

// Rows of a segment rescanned by one wave (16 per lane).
constexpr int kExactWave = 1024;

// Chunks of each candidate's segment, for the candidates found (the scan that
// follows reads no further).
__global__ void k_cand_chunks(const int* __restrict__ cand, const unsigned int* __restrict__ ncand_p,
                              const int* __restrict__ blkseg, const Seg* __restrict__ segs,
                              long long* __restrict__ nch, long long cand_cap) {
  const long long nc = min((long long)*ncand_p, cand_cap);
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += stride) {
    // a segment of at most kExactWave rows is rescanned by a wave of its own
    // (k_exact, first phase) and gets no work items
    const long long n = segs[blkseg[cand[c] >> 4]].n_rows;
    nch[c] = n > kExactWave ? (n + kExactChunk - 1) / kExactChunk : 0;
  }
}

// Exact FP64 rescans of candidate rows.  Work item = (candidate, chunk of its
// segment) from the prefix sum chbase.  PASS 0: maximum squared distance;
// PASS 1: smallest id of the pairs that reach it; PASS 2: smallest partner id
// of those; PASS 3: the rows of the chosen pair (only items whose candidate
// is one of its two vertices scan their chunk).  With ids32 (every id of the
// call below 2^32) PASS 1 takes the smallest id_lo * 2^32 + id_hi at once
// into id_lo, and PASS 2 is not run.
// One candidate row against rows [jb, je) of its segment: the pass's value
// over those pairs, reduced over the lanes that take part (lane, step).
template <int PASS>
__device__ inline unsigned long long exact_scan(long long jb, long long je, int lane, int step, int vi,
                                                const double* pi, unsigned long long idi, const Roi& R,
                                                double target, unsigned long long lo_ref,
                                                unsigned long long hi_ref, int ids32, int g,
                                                const int* __restrict__ orig,
                                                const unsigned long long* __restrict__ key,
                                                const double* __restrict__ tsoft, GroupRes* __restrict__ gres) {
  unsigned long long red = PASS == 0 ? 0ull : ~0ull;
  for (long long j = jb + lane; j < je; j += step) {
    const int vj = orig[j];
    const unsigned long long kj = key[vj];
    double pj[3];
    key_position(kj, tsoft ? tsoft[vj] : 0.5, R.s, pj);
    const double d2 = dist2_exact(pi, pj);
    if (PASS == 0) {
      red = max(red, (unsigned long long)__double_as_longlong(d2));
    } else if (vi != vj && d2 == target) {
      const unsigned long long idj = key_canonical_id(kj, R.d);
      const unsigned long long lo_id = min(idi, idj), hi_id = max(idi, idj);
      if (PASS == 1) red = min(red, ids32 ? (lo_id << 32) | hi_id : lo_id);
      if (PASS == 2 && lo_id == lo_ref) red = min(red, hi_id);
      if (PASS == 3 && lo_id == lo_ref && hi_id == hi_ref) {
        gres[g].row_i = idi == lo_id ? vi : vj;
        gres[g].row_j = idi == lo_id ? vj : vi;
      }
    }
  }
  for (int m = 32; m >= 1; m >>= 1) {
    const unsigned long long o = __shfl_xor(red, m, 64);
    red = PASS == 0 ? max(red, o) : min(red, o);
  }
  return red;
}

template <int PASS>
__device__ inline void exact_commit(GroupRes* __restrict__ gres, int g, unsigned long long red) {
  if (red == (PASS == 0 ? 0ull : ~0ull)) return;
  if (PASS == 0) atomicMax(&gres[g].best_bits, red);
  if (PASS == 1) atomicMin(&gres[g].id_lo, red);
  if (PASS == 2) atomicMin(&gres[g].id_hi, red);
}

// The candidate row, its group and the group's references for the pass.
struct ExactRow {
  int vi, g;
  long long row_begin, n_rows;
  double pi[3];
  unsigned long long idi, lo_ref, hi_ref;
  double target;
};

__device__ inline ExactRow exact_row(int row_i, const int* __restrict__ blkseg, const Seg* __restrict__ segs,
                                     const int* __restrict__ orig, const unsigned long long* __restrict__ key,
                                     const double* __restrict__ tsoft, const Roi* __restrict__ rois,
                                     const GroupRes* __restrict__ gres, int ids32) {
  ExactRow E;
  const Seg S = segs[blkseg[row_i >> 4]];
  E.g = S.group;
  E.row_begin = S.row_begin;
  E.n_rows = S.n_rows;
  const Roi& R = rois[E.g >> 2];
  E.vi = orig[row_i];
  const unsigned long long ki = key[E.vi];
  key_position(ki, tsoft ? tsoft[E.vi] : 0.5, R.s, E.pi);
  E.idi = key_canonical_id(ki, R.d);
  E.target = __longlong_as_double((long long)gres[E.g].best_bits);
  const unsigned long long gl = gres[E.g].id_lo;
  E.lo_ref = ids32 ? gl >> 32 : gl;
  E.hi_ref = ids32 ? gl & 0xffffffffull : gres[E.g].id_hi;
  return E;
}

// Two phases: first every candidate whose segment holds at most kExactWave
// rows, a wave each (most candidates lie in plane buckets of tens to hundreds
// of rows, where a workgroup per candidate would leave most lanes idle and a
// search of chbase per item would cost more than the scan); then the work
// items (candidate, chunk) of the longer segments from the prefix sum
// chbase, a workgroup each.
template <int PASS>
__global__ __launch_bounds__(256) void k_exact(const int* __restrict__ cand, const unsigned int* __restrict__ ncand_p,
                                               const long long* __restrict__ chbase,
                                               const long long* __restrict__ n_work_p,
                                               const int* __restrict__ blkseg, const Seg* __restrict__ segs,
                                               const int* __restrict__ orig, const unsigned long long* __restrict__ key,
                                               const double* __restrict__ tsoft, const Roi* __restrict__ rois,
                                               GroupRes* __restrict__ gres, long long cand_cap, int ids32) {
  __shared__ unsigned long long sh[4];
  const int nc = (int)min((long long)*ncand_p, cand_cap);
  const long long n_work = *n_work_p;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long c = ((long long)blockIdx.x * blockDim.x + tid) >> 6; c < nc; c += nwaves) {
    const int row_i = cand[c];
    if (segs[blkseg[row_i >> 4]].n_rows > kExactWave) continue;
    const ExactRow E = exact_row(row_i, blkseg, segs, orig, key, tsoft, rois, gres, ids32);
    if (PASS == 3 && E.idi != E.lo_ref && E.idi != E.hi_ref) continue;
    const unsigned long long red =
        exact_scan<PASS>(E.row_begin, E.row_begin + E.n_rows, lane, 64, E.vi, E.pi, E.idi, rois[E.g >> 2],
                         E.target, E.lo_ref, E.hi_ref, ids32, E.g, orig, key, tsoft, gres);
    if (PASS != 3 && lane == 0) exact_commit<PASS>(gres, E.g, red);
  }
  for (long long w = blockIdx.x; w < n_work; w += gridDim.x) {
    int lo = 0, hi = nc - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (chbase[mid] <= w)
        lo = mid;
      else
        hi = mid - 1;
    }
    const ExactRow E = exact_row(cand[lo], blkseg, segs, orig, key, tsoft, rois, gres, ids32);
    if (PASS == 3 && E.idi != E.lo_ref && E.idi != E.hi_ref) continue;  // uniform over the workgroup
    const long long jb = E.row_begin + (w - chbase[lo]) * kExactChunk;
    const long long je = min(jb + (long long)kExactChunk, E.row_begin + E.n_rows);
    unsigned long long red = exact_scan<PASS>(jb, je, tid, 256, E.vi, E.pi, E.idi, rois[E.g >> 2], E.target,
                                              E.lo_ref, E.hi_ref, ids32, E.g, orig, key, tsoft, gres);
    if (PASS == 3) continue;
    __syncthreads();
    if (lane == 0) sh[wid] = red;
    __syncthreads();
    if (tid == 0) {
      for (int k = 0; k < 4; ++k) red = PASS == 0 ? max(red, sh[k]) : min(red, sh[k]);
      exact_commit<PASS>(gres, E.g, red);
    }
  }
}

// Also clears the candidate counter, the pair-pass work counters and the row
// maxima of every row the layouts can hold (one launch before the pair pass).
__global__ void k_init_groups(GroupRes* gres, long long n, unsigned int* counters, unsigned int* rowmax_bits,
                              long long n_rows, const long long* __restrict__ totals) {
  if (blockIdx.x == 0) {
    for (int i = kWorkStride + threadIdx.x; i < kCounterWords; i += blockDim.x) counters[i] = 0u;
    if (threadIdx.x == 0) counters[1] = 0u;
  }
  // only the rows laid out by this call (layout 0 and the plane buckets) are
  // written by the pair passes and read after them
  n_rows = min(n_rows, totals[T_ROWS0] + totals[T_ROWS2D]);
  for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < n_rows; r += (long long)gridDim.x * blockDim.x)
    rowmax_bits[r] = 0u;
  for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (long long)gridDim.x * blockDim.x) {
    GroupRes G;
    G.best_bits = 0ull;
    G.id_lo = ~0ull;
    G.id_hi = ~0ull;
    G.row_i = -1;
    G.row_j = -1;
    G.gmax = 0.0f;
    G.n_cand = 0;
    gres[g] = G;
  }
}

// Eigenvalues (ascending) of the symmetric 3x3 matrix with entries
// c = (a00, a11, a22, a01, a02, a12), by cyclic Jacobi rotations (Golub and
// Van Loan, Matrix Computations, Sec. 8.5): each rotation in plane (p, q)
// uses t = sign(th) / (|th| + sqrt(1 + th^2)), th = (a_qq - a_pp) / (2 a_pq),
// the smaller root, which zeroes a_pq; sweeps converge quadratically, and 12
// sweeps leave the off-diagonal entries at rounding level.
__device__ inline void sym3_eigenvalues(const double* c, double* lam) {
  double a[3][3] = {{c[0], c[3], c[4]}, {c[3], c[1], c[5]}, {c[4], c[5], c[2]}};
  for (int sweep = 0; sweep < 12; ++sweep) {
    const double off = fabs(a[0][1]) + fabs(a[0][2]) + fabs(a[1][2]);
    if (off == 0.0) break;
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2, r = 3 - p - q;
      const double apq = a[p][q];
      if (apq == 0.0) continue;
      const double th = (a[q][q] - a[p][p]) / (2.0 * apq);
      const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
      const double cs = 1.0 / sqrt(1.0 + t * t), sn = t * cs;
      a[p][p] -= t * apq;
      a[q][q] += t * apq;
      a[p][q] = a[q][p] = 0.0;
      const double arp = a[r][p], arq = a[r][q];
      a[r][p] = a[p][r] = cs * arp - sn * arq;
      a[r][q] = a[q][r] = sn * arp + cs * arq;
    }
  }
  double e0 = a[0][0], e1 = a[1][1], e2 = a[2][2], tmp;
  if (e0 > e1) { tmp = e0; e0 = e1; e1 = tmp; }
  if (e1 > e2) { tmp = e1; e1 = e2; e2 = tmp; }
  if (e0 > e1) { tmp = e0; e0 = e1; e1 = tmp; }
  lam[0] = e0;
  lam[1] = e1;
  lam[2] = e2;
}

// The Shape-class members that follow from MeshVolume V, SurfaceArea A, the
// inside-voxel count and the covariance eigenvalues (PyRadiomics' Shape class
// definitions): VoxelVolume, SurfaceVolumeRatio, Sphericity, Compactness1,
// Compactness2, SphericalDisproportion, Major/Minor/LeastAxisLength (4 sqrt
// of the largest, middle and smallest eigenvalue, negative rounding clamped
// to 0), Elongation and Flatness (0 when the largest eigenvalue is 0).
__device__ inline void shape_class_members(const RoiMeta& M, const Roi& R, double V, double A, double* f) {
  const double pi = 3.14159265358979323846;
  f[0] = (double)M.n_in * (R.s[0] * R.s[1] * R.s[2]);
  f[1] = A / V;
  const double k = cbrt(36.0 * pi * V * V);
  f[2] = k / A;
  f[3] = V / (sqrt(pi) * A * sqrt(A));
  f[4] = 36.0 * pi * V * V / (A * A * A);
  f[5] = A / k;
  double lam[3];
  sym3_eigenvalues(M.cov, lam);
  for (int i = 0; i < 3; ++i) lam[i] = lam[i] > 0.0 ? lam[i] : 0.0;
  f[6] = 4.0 * sqrt(lam[2]);
  f[7] = 4.0 * sqrt(lam[1]);
  f[8] = 4.0 * sqrt(lam[0]);
  f[9] = lam[2] > 0.0 ? sqrt(lam[1] / lam[2]) : 0.0;
  f[10] = lam[2] > 0.0 ? sqrt(lam[0] / lam[2]) : 0.0;
}

__global__ void k_finalize(int n_rois, const RoiMeta* __restrict__ meta, const GroupRes* __restrict__ gres,
                           const unsigned int* __restrict__ ncand, const unsigned long long* __restrict__ key,
                           const Roi* __restrict__ rois, const long long* __restrict__ pairs2d,
                           RoiResult* __restrict__ res, long long cand_cap, int moments, int ids32) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n_rois; r += gridDim.x * blockDim.x) {
    const RoiMeta M = meta[r];
    RoiResult Q;
    Q.V = M.V;
    Q.T = M.T;
    Q.pairs2d = pairs2d[r];
    Q.out[0] = fabs(M.vol);
    Q.vol_signed = M.vol;
    Q.out[1] = M.area;
    for (int f = 0; f < 4; ++f) {
      const GroupRes G = gres[4 * r + f];
      const double d2 = __longlong_as_double((long long)G.best_bits);
      Q.out[2 + f] = sqrt(d2);
      const bool have = G.id_lo != ~0ull;
      const unsigned long long lo = ids32 ? G.id_lo >> 32 : G.id_lo, hi = ids32 ? G.id_lo & 0xffffffffull : G.id_hi;
      Q.ids[f][0] = have ? (long long)lo : -1;
      Q.ids[f][1] = have ? (long long)hi : -1;
      Q.rows[f][0] = have ? G.row_i : -1;
      Q.rows[f][1] = have ? G.row_j : -1;
      Q.cand[f] = G.n_cand;
    }
    Q.status = M.V == 0 ? 1 : 0;
    if ((long long)*ncand > cand_cap || ncand[1] != 0u) Q.status = -4;
    if (rois[r].status != 0) Q.status = rois[r].status;
    Q.pad_ = 0;
    Q.n_in = moments ? M.n_in : 0;
    for (int f = 0; f < 11; ++f) Q.shape[f] = 0.0;
    if (moments && Q.status == 0) shape_class_members(M, rois[r], Q.out[0], Q.out[1], Q.shape);
    res[r] = Q;
  }
}

// Per-ROI results to the caller's device arrays: out[nf r .. nf r + nf - 1]
// (the six features, then with nf = 17 the other Shape-class members; left
// untouched for a negative status) and status[r].
__global__ void k_results_out(const RoiResult* __restrict__ res, int n_rois, double* __restrict__ out,
                              int* __restrict__ status, int nf) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n_rois; r += gridDim.x * blockDim.x) {
    const int st = res[r].status;
    if (st >= 0) {
      for (int f = 0; f < 6; ++f) out[(long long)nf * r + f] = res[r].out[f];
      for (int f = 6; f < nf; ++f) out[(long long)nf * r + f] = res[r].shape[f - 6];
    }
    if (status) status[r] = st;
  }
}

__global__ void k_export_vertices(const unsigned long long* __restrict__ key, const double* __restrict__ tsoft,
                                  const Roi* __restrict__ rois, long long V, long long* __restrict__ ids,
                                  double* __restrict__ pos) {
  const Roi R = rois[0];
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += (long long)gridDim.x * blockDim.x) {
    ids[v] = (long long)key_canonical_id(key[v], R.d);
    if (pos) {
      double x[3];
      key_position(key[v], tsoft ? tsoft[v] : 0.5, R.s, x);
      pos[3 * v] = x[0];
      pos[3 * v + 1] = x[1];
      pos[3 * v + 2] = x[2];
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers.

static unsigned grid_for(long long n, long long cap = 8192) {
  long long g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// Whether small plane buckets go to k_pair_small_h: split-f16 kernel, and
// enough buckets that the extra launch (about 15 us on a single small ROI)
// is paid back by the work-list items it saves (about 1 ms on 4,096 ROIs).
static bool small_buckets(const PairBufs& B) { return B.tune.kernel == 1 && B.n_buckets >= kSmallMinBuckets; }

// The split-f16 operand rows when the pair pass runs kernel 1 (then they are
// written in place of the FP32 positions), else null.
uint4* split_rows(const PairBufs& B) { return B.tune.kernel == 1 ? B.posh : nullptr; }

static BrickArgs brick_args(const PairBufs& B) {
  BrickArgs A;
  A.rois = B.rois;
  A.n_rois = B.n_rois;
  A.meta = B.meta;
  A.part = B.part;
  A.brick_voff = B.brick_voff;
  A.bmap = B.n_rois > 1 ? B.bmap : nullptr;
  A.nbricks = B.nbricks;
  return A;
}

hipError_t launch_buckets(const PairBufs& B, hipStream_t st) {
  hipError_t e;
  // Whole plane buckets are pruned with the pair tiles in calls with many
  // buckets: their boxes cost the histogram pass four more atomics per group
  // of lanes, which the pruned scatter and pair work repay on a batch of
  // small ROIs (4,096 ROIs: 19.3 -> 19.0 ms) but not on one large ROI
  // (2,651 buckets: 0.83 -> 0.95 ms).
  int4* bbox = B.prune && B.n_buckets >= kSmallMinBuckets ? B.bbox : nullptr;
  hipLaunchKernelGGL(k_zero_buckets, dim3(grid_for(std::max<long long>(B.n_buckets, B.n_rois), 4096)), dim3(256), 0,
                     st, B.bcnt, B.bcur, B.n_buckets, B.pairs2d, (long long)B.n_rois, bbox);
  const BrickArgs A = brick_args(B);
  if (B.nbricks > 0)
    hipLaunchKernelGGL(k_brick_hist, dim3((unsigned)B.nbricks), dim3(256), sizeof(int) * B.brick_win * (bbox ? 5 : 1),
                       st, A, B.key, B.bcnt, bbox, B.brick_win);
  if (bbox)
    hipLaunchKernelGGL(k_bucket_prune, dim3((unsigned)B.n_rois), dim3(256), 0, st, B.rois, B.tsoft ? 1 : 0, B.bcnt,
                       bbox, B.pairs2d);
  hipLaunchKernelGGL(k_bucket_sizes, dim3(grid_for(B.n_buckets)), dim3(256), 0, st, B.bcnt, B.n_buckets, B.bsz,
                     B.bflag);
  if ((e = launch_scan(B.bsz, B.brow, B.n_buckets, B.totals + T_ROWS2D, B.scan_tmp, st))) return e;
  if ((e = launch_scan(B.bflag, B.bseg, B.n_buckets, B.totals + T_NSEG2D, B.scan_tmp, st))) return e;
  if (B.nbricks > 0)
    hipLaunchKernelGGL(k_brick_scatter, dim3((unsigned)B.nbricks), dim3(256),
                       sizeof(int) * (2 * B.brick_win + kScatterList), st, A,
                       B.key, B.totals, B.bcnt, B.bcur, B.brow, B.pos, split_rows(B), B.orig, B.brick_win);
  hipLaunchKernelGGL(k_bucket_groups, dim3((unsigned)B.n_rois), dim3(256), 0, st, B.rois, B.bgroup, B.bcnt,
                     B.pairs2d);
  {
    const int per_wave = B.n_buckets >= kSmallMinBuckets ? 64 : 1;
    hipLaunchKernelGGL(k_bucket_segs, dim3(grid_for(64 * B.n_buckets / per_wave)), dim3(256), 0, st, B.bgroup,
                       B.n_rois, B.n_buckets, B.totals, B.bcnt, B.bsz, B.brow, B.bseg, B.pos, split_rows(B), B.orig,
                       B.blkseg, B.segs, per_wave);
  }
  hipLaunchKernelGGL(k_seg_cols, dim3(grid_for(std::max(B.seg_cap, B.col_cap))), dim3(256), 0, st, B.n_rois,
                     B.seg_cap, B.totals, B.segs, B.meta, B.ncol, B.tune.jchunk,
                     small_buckets(B) ? kSmallBlocks * 32 : 0, B.nitem, B.col_cap, B.prune ? 1 : 0, B.prune_min_v,
                     B.counters);
  if ((e = launch_scan(B.ncol, B.colbase, B.seg_cap, B.totals + T_NCOL, B.scan_tmp, st))) return e;
  hipLaunchKernelGGL(k_col_fill, dim3(grid_for(B.seg_cap)), dim3(256), 0, st, B.n_rois, B.seg_cap, B.totals, B.segs,
                     B.meta, B.ncol, B.colbase, B.cols, B.nitem, B.tune.itile, B.tune.jchunk);
  if ((e = launch_scan(B.nitem, B.itembase, B.col_cap, B.totals + T_NITEM, B.scan_tmp, st))) return e;
  return hipGetLastError();
}

// The work counters (B.counters + kWorkStride) must be zero when this is enqueued.
template <int IT>
hipError_t launch_pair_maxima_it(const PairBufs& B, hipStream_t st) {
  hipError_t e;
  int per_cu = 0;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pair_maxima<IT>, 256, 0))) return e;
  if (per_cu < 1) per_cu = 1;
  if (B.tune.blocks_per_cu > 0 && B.tune.blocks_per_cu < per_cu) per_cu = B.tune.blocks_per_cu;
  const unsigned grid = (unsigned)(B.cu_count * per_cu);
  hipLaunchKernelGGL(k_pair_maxima<IT>, dim3(grid), dim3(256), 0, st, B.pos, B.cols, B.itembase, B.totals,
                     B.counters + kWorkStride, B.rowmax, B.tune.jchunk);
  return hipGetLastError();
}

template <int IT>
hipError_t launch_pair_maxima_h(const PairBufs& B, hipStream_t st) {
  hipError_t e;
  int per_cu = 0;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pair_maxima_h<IT>, 256, 0))) return e;
  if (per_cu < 1) per_cu = 1;
  if (B.tune.blocks_per_cu > 0 && B.tune.blocks_per_cu < per_cu) per_cu = B.tune.blocks_per_cu;
  const unsigned grid = (unsigned)(B.cu_count * per_cu);
  if (B.prune) {
    int per = 0;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_pair_list_h<IT>, 256, 0))) return e;
    if (per < 1) per = 1;
    hipLaunchKernelGGL(k_pair_list_h<IT>, dim3((unsigned)(B.cu_count * per)), dim3(256), 0, st, B.posh, B.pitems,
                       B.counters, B.pitem_cap, B.counters + kListCounters, B.rowmax);
  }
  hipLaunchKernelGGL(k_pair_maxima_h<IT>, dim3(grid), dim3(256), 0, st, B.posh, B.cols, B.itembase, B.totals,
                     B.counters + kWorkStride, B.rowmax, B.tune.jchunk);
  // small plane buckets (bucket count bounded by n_buckets on the host), in
  // tiles of two row blocks: 124 VGPRs, four waves per SIMD for this
  // latency-bound kernel
  const long long waves = (B.n_buckets + kSmallPerWave - 1) / kSmallPerWave;
  if (small_buckets(B) && waves > 0)
    hipLaunchKernelGGL(k_pair_small_h<2>, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, B.posh, B.segs,
                       B.n_rois, B.totals, B.meta, B.rowmax);
  return hipGetLastError();
}

hipError_t launch_pair_maxima(const PairBufs& B, hipStream_t st) {
  if (B.tune.kernel == 1) {
    switch (B.tune.itile) {
      case 4:
        return launch_pair_maxima_h<2>(B, st);
      case 8:
        return launch_pair_maxima_h<4>(B, st);
      default:
        return hipErrorInvalidValue;
    }
  }
  switch (B.tune.itile) {
    case 2:
      return launch_pair_maxima_it<2>(B, st);
    case 4:
      return launch_pair_maxima_it<4>(B, st);
    case 8:
      return launch_pair_maxima_it<8>(B, st);
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_init_groups(const PairBufs& B, hipStream_t st) {
  hipLaunchKernelGGL(k_init_groups, dim3(grid_for(std::max<long long>(4ll * B.n_rois, B.rows_bound), 4096)), dim3(256), 0,
                     st, B.gres, 4ll * B.n_rois, B.counters, (unsigned int*)B.rowmax, B.rows_bound, B.totals);
  return hipGetLastError();
}

hipError_t launch_refine(const PairBufs& B, hipStream_t st) {
  hipError_t e;
  // about 8 chunks of 64 blocks per wave (a few waves per group on one large ROI)
  hipLaunchKernelGGL(k_group_max, dim3(grid_for(B.rows_bound / kBlk / 8, 1024)), dim3(256), 0, st, B.rowmax, B.blkseg,
                     B.segs, B.totals, B.gres);
  hipLaunchKernelGGL(k_candidates, dim3(grid_for(B.rows_bound / kBlk)), dim3(256), 0, st, B.rowmax, B.blkseg, B.segs,
                     B.meta, B.totals, B.gres, B.counters + 1, B.cand, B.cand_cap,
                     B.tune.kernel == 1 ? 6.103515625e-05 /* 2^-14 */ : 7.62939453125e-06 /* 2^-17 */);
  hipLaunchKernelGGL(k_cand_chunks, dim3(grid_for(B.cand_cap)), dim3(256), 0, st, B.cand, B.counters + 1, B.blkseg,
                     B.segs, B.cand_nch, B.cand_cap);
  if ((e = launch_scan(B.cand_nch, B.cand_chbase, B.cand_cap, B.totals + T_NEXACT, B.scan_tmp, st, B.counters + 1)))
    return e;
  const unsigned grid = (unsigned)(B.cu_count * 8);
#define S3D_EXACT(P)                                                                                             \
  hipLaunchKernelGGL(k_exact<P>, dim3(grid), dim3(256), 0, st, B.cand, B.counters + 1, B.cand_chbase,             \
                     B.totals + T_NEXACT, B.blkseg, B.segs, B.orig, B.key, B.tsoft, B.rois, B.gres, B.cand_cap,    \
                     B.ids32 ? 1 : 0)
  S3D_EXACT(0);
  S3D_EXACT(1);
  if (!B.ids32) S3D_EXACT(2);
  S3D_EXACT(3);
#undef S3D_EXACT
  return hipGetLastError();
}

hipError_t launch_finalize(const PairBufs& B, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(grid_for(B.n_rois)), dim3(256), 0, st, B.n_rois, B.meta, B.gres,
                     B.counters + 1, B.key, B.rois, B.pairs2d, B.res, B.cand_cap, B.moments ? 1 : 0, B.ids32 ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_results_out(const RoiResult* res, int n_rois, double* out, int* status, int nf, hipStream_t st) {
  hipLaunchKernelGGL(k_results_out, dim3(grid_for(n_rois, 1024)), dim3(256), 0, st, res, n_rois, out, status, nf);
  return hipGetLastError();
}

hipError_t launch_export_vertices(const unsigned long long* key, const double* tsoft, const RoiMeta* meta,
                                  const Roi* rois, long long* ids, double* pos, long long V, hipStream_t st) {
  (void)meta;
  if (V <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_export_vertices, dim3(grid_for(V)), dim3(256), 0, st, key, tsoft, rois, V, ids, pos);
  return hipGetLastError();
}

}  // namespace s3d
