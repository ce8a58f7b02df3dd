// small.hip -- the single-ROI path for small meshes: after the mesh pass, two
// persistent kernels evaluate every vertex pair exactly in FP64 (the four
// diameters at once) and the last workgroup of the second assembles the
// ROI's result.
//
// For a mesh of a few thousand vertices the general pipeline (plane buckets,
// work lists, the matrix-core filter, candidate refinement: some thirty
// launches and a read-back of the vertex count) costs far more than the pairs
// themselves: 8,000 vertices make 3.2e7 pairs, a few hundred million FP64
// operations, tens of microseconds of the chip.  The diameters (Sec. 2,
// parallel diameter calculation) are the maxima of the exact FP64 squared
// distances over all pairs, and over the pairs that share a plane key for the
// planar ones, with the lexicographically smallest (id_i, id_j) among ties:
// the first kernel takes the four maxima (a max per pair, no branches), the
// second the smallest id pair among the pairs at each maximum (pairs equal to
// a maximum are rare, so it rarely branches either).  The distances are the
// same FP64 operations as the general path's exact refinement, so the
// results are identical.  The area and volume of binary masks follow from
// integers (case counts, volume units); soft masks' brick partials are summed
// in the general path's order, with the general path's bricks.
#include <algorithm>

#include "s3d_device.h"
#include "s3d_launch.h"

namespace s3d {

namespace {

constexpr int kTile = 128;  // rows and columns of a pair tile

// A staged column of a tile: FP64 position, canonical id and plane keys.
struct ColRec {
  double x[3];
  unsigned long long id;
  int pk[3];
  int pad_;
};

// The plane keys of a vertex (its coordinate along each axis in half voxels).
__device__ inline void plane_keys(unsigned long long k, int* pk) {
  const int a = (int)((k >> 60) & 3);
  pk[0] = 2 * ((int)((k >> 40) & 0xFFFFF) - 1) + (a == 0);
  pk[1] = 2 * ((int)((k >> 20) & 0xFFFFF) - 1) + (a == 1);
  pk[2] = 2 * ((int)(k & 0xFFFFF) - 1) + (a == 2);
}

// Tile t of the upper triangle of nb x nb tiles, numbered row by row (the
// rows before row b hold b nb - b (b - 1) / 2 tiles).
__device__ inline void tile_coords(long long t, long long nb, long long& bi, long long& bj) {
  const double q = (double)(2 * nb + 1);
  bi = (long long)((q - sqrt(q * q - 8.0 * (double)t)) * 0.5);
  while (bi > 0 && bi * nb - bi * (bi - 1) / 2 > t) --bi;
  while ((bi + 1) * nb - (bi + 1) * bi / 2 <= t) ++bi;
  bj = bi + (t - (bi * nb - bi * (bi - 1) / 2));
}

// The staged vertex count the pair kernels work on (0 when the mesh did not fit).
__device__ inline long long small_v(const long long* totals, long long vmax) {
  const long long staged = totals[8];
  return staged <= vmax ? staged : 0;
}

// A row of a tile held in registers.
struct RowRec {
  double x[3];
  unsigned long long id;
  int pk[3];
  bool ok;  // the row is a vertex (rows past the last one occur in the last diagonal tile only)
};

// Stages the tile's columns in LDS and loads this thread's two rows (lane
// and lane + 64 of the tile's row block).
__device__ inline void stage_tile(const Roi& R, const unsigned long long* tmpkey, const double* tmpt, long long V,
                                  long long bi, long long bj, ColRec* s_col, RowRec* row) {
  __syncthreads();  // the previous tile's columns are no longer read
  if (threadIdx.x < kTile) {
    const long long j = bj * kTile + threadIdx.x;
    if (j < V) {
      const unsigned long long k = tmpkey[j];
      ColRec C;
      key_position(k, tmpt ? tmpt[j] : 0.5, R.s, C.x);
      C.id = key_canonical_id(k, R.d);
      plane_keys(k, C.pk);
      C.pad_ = 0;
      s_col[threadIdx.x] = C;
    }
  }
  for (int h = 0; h < 2; ++h) {
    const long long i = bi * kTile + (threadIdx.x & 63) + 64 * h;
    row[h].ok = i < V;
    const unsigned long long k = tmpkey[row[h].ok ? i : 0];
    key_position(k, tmpt ? tmpt[row[h].ok ? i : 0] : 0.5, R.s, row[h].x);
    row[h].id = key_canonical_id(k, R.d);
    plane_keys(k, row[h].pk);
  }
  __syncthreads();
}

// Column range of a wave within a tile: a quarter of the columns each.
__device__ inline void wave_cols(long long V, long long bj, int& c0, int& c1) {
  const int ncols = (int)min((long long)kTile, V - bj * kTile);
  c0 = (threadIdx.x >> 6) * (kTile / 4);
  c1 = min(c0 + kTile / 4, ncols);
}

}  // namespace

// Pass 1, persistent over the pair tiles (bi <= bj, kTile x kTile) of the
// staged vertices: the four maximum squared distances (3D, then the planes of
// axes 0, 1, 2) into acc->gmax (as FP64 bits; non-negative doubles order as
// their bits), the in-plane pair count into acc->pairs2d, and each wave's
// four maxima of each tile into tmax[(t * 4 + wave) * 4 + group] (-1 where
// the wave had no pair of the group).  A thread
// holds two rows of a tile (lane, lane + 64) in registers; each wave takes a
// quarter of the tile's columns, staged in LDS, so all its lanes read the
// same column and each column read serves two pairs.  The loop bodies are
// straight-line code: every test is evaluated, none short-circuits.
__global__ __launch_bounds__(256) void k_small_max(const Roi* __restrict__ rois,
                                                   const unsigned long long* __restrict__ tmpkey,
                                                   const double* __restrict__ tmpt,
                                                   const long long* __restrict__ totals, long long vmax,
                                                   SmallAcc* __restrict__ acc, double* __restrict__ tmax) {
  __shared__ ColRec s_col[kTile];
  __shared__ double s_m[4][4];
  __shared__ long long s_p2[4];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const Roi R = rois[0];
  const long long V = small_v(totals, vmax);
  const long long nb = (V + kTile - 1) / kTile;
  const long long ntiles = nb * (nb + 1) / 2;
  double m[4] = {0.0, 0.0, 0.0, 0.0};
  long long p2 = 0;  // this wave's in-plane pairs (wave-uniform)
  for (long long t = blockIdx.x; t < ntiles; t += gridDim.x) {
    long long bi, bj;
    tile_coords(t, nb, bi, bj);
    RowRec row[2];
    stage_tile(R, tmpkey, tmpt, V, bi, bj, s_col, row);
    int c0, c1;
    wave_cols(V, bj, c0, c1);
    // this tile's maxima of the wave; -1 while the wave has no pair of the group
    double tm[4] = {-1.0, -1.0, -1.0, -1.0};
    if (bi != bj) {
      // every pair of the tile counts
      for (int c = c0; c < c1; ++c) {
        const ColRec C = s_col[c];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const double d = dist2_exact(row[h].x, C.x);
          const bool e0 = row[h].pk[0] == C.pk[0];
          const bool e1 = row[h].pk[1] == C.pk[1];
          const bool e2 = row[h].pk[2] == C.pk[2];
          p2 += __popcll(__ballot(e0)) + __popcll(__ballot(e1)) + __popcll(__ballot(e2));
          tm[0] = fmax(tm[0], d);
          tm[1] = fmax(tm[1], e0 ? d : -1.0);
          tm[2] = fmax(tm[2], e1 ? d : -1.0);
          tm[3] = fmax(tm[3], e2 ? d : -1.0);
        }
      }
    } else {
      // the diagonal tile: only columns after the row, and rows that exist
      for (int c = c0; c < c1; ++c) {
        const ColRec C = s_col[c];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const bool valid = (c > lane + 64 * h) & row[h].ok;
          const double dd = dist2_exact(row[h].x, C.x);
          const double d = valid ? dd : -1.0;
          const bool e0 = valid & (row[h].pk[0] == C.pk[0]);
          const bool e1 = valid & (row[h].pk[1] == C.pk[1]);
          const bool e2 = valid & (row[h].pk[2] == C.pk[2]);
          p2 += __popcll(__ballot(e0)) + __popcll(__ballot(e1)) + __popcll(__ballot(e2));
          tm[0] = fmax(tm[0], d);
          tm[1] = fmax(tm[1], e0 ? d : -1.0);
          tm[2] = fmax(tm[2], e1 ? d : -1.0);
          tm[3] = fmax(tm[3], e2 ? d : -1.0);
        }
      }
    }
    for (int g = 0; g < 4; ++g) {
      for (int k = 32; k >= 1; k >>= 1) tm[g] = fmax(tm[g], __shfl_xor(tm[g], k, 64));
      m[g] = fmax(m[g], tm[g]);
    }
    if (lane < 4) tmax[(t * 4 + wid) * 4 + lane] = tm[0] * (lane == 0) + tm[1] * (lane == 1) +
                                                     tm[2] * (lane == 2) + tm[3] * (lane == 3);
  }
  if (lane == 0) {
    for (int g = 0; g < 4; ++g) s_m[g][wid] = m[g];
    s_p2[wid] = p2;
  }
  __syncthreads();
  if (tid < 4) {
    const double v = fmax(fmax(s_m[tid][0], s_m[tid][1]), fmax(s_m[tid][2], s_m[tid][3]));
    if (v > 0.0) atomicMax(&acc->gmax[tid], (unsigned long long)__double_as_longlong(v));
  } else if (tid == 4) {
    const long long n = s_p2[0] + s_p2[1] + s_p2[2] + s_p2[3];
    if (n) atomicAdd(&acc->pairs2d, (unsigned long long)n);
  }
}

// Pass 2: among the pairs whose squared distance equals a group's maximum,
// the smallest (id_lo, id_hi), packed as id_lo * 2^32 + id_hi (ids of a
// small ROI stay below 2^32), into acc->key; only the tiles where some wave
// reached a group's maximum are visited again.  The last workgroup to finish
// (acc->ticket) sums the bricks and writes the ROI's result.  More than vmax
// staged vertices: status kSmallOverflow (the caller then runs the general
// path).
__global__ __launch_bounds__(256) void k_small_pick(const Roi* __restrict__ rois, const BrickPart* __restrict__ part,
                                                    long long nbricks, const double* __restrict__ case_area,
                                                    const unsigned long long* __restrict__ tmpkey,
                                                    const double* __restrict__ tmpt,
                                                    const long long* __restrict__ totals, long long vmax,
                                                    const double* __restrict__ tmax, SmallAcc* __restrict__ acc,
                                                    RoiResult* __restrict__ res, int dtype) {
  __shared__ ColRec s_col[kTile];
  __shared__ unsigned long long s_k[4][4];
  __shared__ double s_d[2][256];
  __shared__ long long s_l[3][4];
  __shared__ bool s_last;
  __shared__ int s_hit;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const Roi R = rois[0];
  const long long V = small_v(totals, vmax);
  const long long nb = (V + kTile - 1) / kTile;
  const long long ntiles = nb * (nb + 1) / 2;
  unsigned long long gm[4];
  for (int g = 0; g < 4; ++g) gm[g] = acc->gmax[g];
  unsigned long long key[4] = {~0ull, ~0ull, ~0ull, ~0ull};
  for (long long t = blockIdx.x; t < ntiles; t += gridDim.x) {
    __syncthreads();
    if (tid == 0) s_hit = 0;
    __syncthreads();
    if (tid < 16 && (unsigned long long)__double_as_longlong(tmax[t * 16 + tid]) == gm[tid & 3]) s_hit = 1;
    __syncthreads();
    if (!s_hit) continue;
    long long bi, bj;
    tile_coords(t, nb, bi, bj);
    RowRec row[2];
    stage_tile(R, tmpkey, tmpt, V, bi, bj, s_col, row);
    int c0, c1;
    wave_cols(V, bj, c0, c1);
    const bool diag = bi == bj;
    for (int c = c0; c < c1; ++c) {
      const ColRec C = s_col[c];
      for (int h = 0; h < 2; ++h) {
        const bool valid = !diag | ((c > lane + 64 * h) & row[h].ok);
        const unsigned long long d2 = (unsigned long long)__double_as_longlong(dist2_exact(row[h].x, C.x));
        const bool t0 = valid & (d2 == gm[0]);
        const bool t1 = valid & (d2 == gm[1]) & (row[h].pk[0] == C.pk[0]);
        const bool t2 = valid & (d2 == gm[2]) & (row[h].pk[1] == C.pk[1]);
        const bool t3 = valid & (d2 == gm[3]) & (row[h].pk[2] == C.pk[2]);
        if (t0 | t1 | t2 | t3) {
          const unsigned long long lo = min(row[h].id, C.id), hi = max(row[h].id, C.id);
          const unsigned long long k = (lo << 32) | hi;
          if (t0) key[0] = min(key[0], k);
          if (t1) key[1] = min(key[1], k);
          if (t2) key[2] = min(key[2], k);
          if (t3) key[3] = min(key[3], k);
        }
      }
    }
  }
  for (int g = 0; g < 4; ++g)
    for (int k = 32; k >= 1; k >>= 1) key[g] = min(key[g], (unsigned long long)__shfl_xor(key[g], k, 64));
  if (lane == 0)
    for (int g = 0; g < 4; ++g) s_k[g][wid] = key[g];
  __syncthreads();
  if (tid < 4) {
    const unsigned long long v = min(min(s_k[tid][0], s_k[tid][1]), min(s_k[tid][2], s_k[tid][3]));
    if (v != ~0ull) atomicMin(&acc->key[tid], v);
  }
  __syncthreads();
  if (tid == 0) {
    __threadfence();
    s_last = atomicAdd(&acc->ticket, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();

  // --- the last workgroup: integer totals (any order), soft area and volume
  // in the general path's order (1,024 contiguous brick chunks, then a
  // halving tree; its first two levels stay within a thread here)
  const long long n = nbricks;
  const long long chunk = (n + 1023) / 1024;
  long long nv = 0, nt = 0, vi = 0;
  double a4[4], v4[4];
  for (int q = 0; q < 4; ++q) {
    const int v = tid + 256 * q;
    const long long lo = min(n, chunk * v), hi = min(n, chunk * (v + 1));
    double area = 0.0, vd = 0.0;
    for (long long b = lo; b < hi; ++b) {
      const BrickPart P = part[b];
      nv += P.nv;
      nt += P.nt;
      vi += P.vol_i;
      area += P.area;
      vd += P.vol_d;
    }
    a4[q] = area;
    v4[q] = vd;
  }
  // level 512: v += v + 512 (v = tid, tid + 256); level 256: v += v + 256
  a4[0] += a4[2];
  a4[1] += a4[3];
  v4[0] += v4[2];
  v4[1] += v4[3];
  s_d[0][tid] = a4[0] + a4[1];
  s_d[1][tid] = v4[0] + v4[1];
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (tid < w) {
      s_d[0][tid] += s_d[0][tid + w];
      s_d[1][tid] += s_d[1][tid + w];
    }
    __syncthreads();
  }
  if (dtype == 0) binary_area_tree(case_area, case_hist(case_area, 1), s_d[0]);  // s_d[0] is free for binary masks
  nv = wave_sum(nv);
  nt = wave_sum(nt);
  vi = wave_sum(vi);
  if (lane == 0) {
    s_l[0][wid] = nv;
    s_l[1][wid] = nt;
    s_l[2][wid] = vi;
  }
  __syncthreads();
  if (tid == 0) {
    const long long Vt = s_l[0][0] + s_l[0][1] + s_l[0][2] + s_l[0][3];
    const long long Tt = s_l[1][0] + s_l[1][1] + s_l[1][2] + s_l[1][3];
    const long long Vi = s_l[2][0] + s_l[2][1] + s_l[2][2] + s_l[2][3];
    RoiResult Q;
    const double vol = dtype == 0 ? (double)Vi * (R.s[0] * R.s[1] * R.s[2] / 48.0) : s_d[1][0];
    Q.V = Vt;
    Q.T = Tt;
    Q.out[0] = fabs(vol);
    Q.vol_signed = vol;
    Q.out[1] = s_d[0][0];
    Q.pairs2d = (long long)acc->pairs2d;
    for (int g = 0; g < 4; ++g) {
      const unsigned long long k = acc->key[g];
      Q.out[2 + g] = sqrt(__longlong_as_double((long long)acc->gmax[g]));
      const bool have = k != ~0ull;
      Q.ids[g][0] = have ? (long long)(k >> 32) : -1;
      Q.ids[g][1] = have ? (long long)(k & 0xFFFFFFFFull) : -1;
      Q.rows[g][0] = -1;
      Q.rows[g][1] = -1;
      Q.cand[g] = 0;
    }
    Q.status = Vt == 0 ? 1 : 0;
    if (totals[8] > vmax) Q.status = kSmallOverflow;
    Q.n_in = 0;
    for (int f = 0; f < 11; ++f) Q.shape[f] = 0.0;
    Q.pad_ = 0;
    res[0] = Q;
  }
}

size_t small_acc_bytes() {
  const long long nb = (kSmallMaxV + kTile - 1) / kTile;
  return 256 + sizeof(double) * 16 * (size_t)(nb * (nb + 1) / 2);
}

hipError_t launch_small_pairs(int dtype, const Roi* rois, const BrickPart* part, long long nbricks,
                              const double* case_area, const unsigned long long* tmpkey, const double* tmpt,
                              const long long* totals, long long vmax, SmallAcc* acc, int n_groups,
                              RoiResult* res, hipStream_t st) {
  static_assert(sizeof(SmallAcc) <= 256, "the tile maxima follow the accumulators");
  double* tmax = (double*)((char*)acc + 256);
  hipLaunchKernelGGL(k_small_max, dim3((unsigned)n_groups), dim3(256), 0, st, rois, tmpkey, tmpt, totals, vmax, acc,
                     tmax);
  // the second pass mostly checks tile maxima: a quarter of the workgroups
  hipLaunchKernelGGL(k_small_pick, dim3((unsigned)std::max(1, n_groups / 4)), dim3(256), 0, st, rois, part, nbricks,
                     case_area,
                     tmpkey, tmpt, totals, vmax, (const double*)tmax, acc, res, dtype);
  return hipGetLastError();
}

}  // namespace s3d
