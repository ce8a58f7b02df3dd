// soft.hip -- adjoint of the soft-mask (probability) forward pass.
//
// L = sum_f g_f F_f over the six features.  The vertex on crossing edge
// (u, u + e_a) sits at x = (u + t e_a) * s with t = (0.5 - p_u) / (p_b - p_u), so
//   dL/dp_w = sum over crossing edges incident to voxel w of
//             (dL/dx_v)_a * s_a * dt/dp_w,
//   dt/dp_u = (0.5 - p_b) / (p_b - p_u)^2,  dt/dp_b = -(0.5 - p_u) / (p_b - p_u)^2.
// dL/dx_v gathers, over the triangles of the four cubes around the edge that
// contain v (a the vertex, b and c the next ones in the triangle's order):
//   area:   g_area * 1/2 * nhat x (c - b)
//   volume: g_vol * sign(SV) * (b' x c') / 6   (primes: relative to the array
//           centre, the origin of the signed sum)
// plus the diameter subgradient g_f (x_v - x_other) / D_f when v is an end
// point of the maximising pair of feature f.
//
// Three passes over every ROI of a table:
//   1. k_soft_edges: one wave per padded cube row lists the row's crossing
//      edges (their slots in the edge field); a workgroup reserves room for
//      its rows with one atomic;
//   2. k_soft_vertex_grad: one thread per crossing edge (the surface is sparse,
//      so a thread per voxel would leave most lanes idle around the FP64 work)
//      computes (dL/dx_v)_a * s_a into the edge's field slot;
//   3. k_soft_gather: one wave per voxel row sums, for each voxel, the terms of
//      its (at most six) incident crossing edges, read directly from their
//      field slots, and writes dL/dp densely (0 away from the surface).
// Only slots of crossing edges are written and read, so the field is never
// cleared.  No float atomics: the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#define MC_TABLE_QUAL __constant__ const
#include "mc_table.h"
#include "s3d_device.h"
#include "s3d_launch.h"

namespace s3d {

__device__ inline double pval(const float* p, const int* d, int z, int y, int x) {
  if (z < 0 || y < 0 || x < 0 || z >= d[0] || y >= d[1] || x >= d[2]) return 0.0;
  return (double)p[((size_t)z * d[1] + y) * (size_t)d[2] + x];
}

// Position (relative to the origin o) of the vertex on the edge from voxel u
// along axis a.
__device__ inline void vertex_pos(const float* p, const int* d, const double* s, const double* o, int u0, int u1,
                                  int u2, int a, double* x) {
  const double pa = pval(p, d, u0, u1, u2);
  const double pb = pval(p, d, u0 + (a == 0), u1 + (a == 1), u2 + (a == 2));
  const double t = (0.5 - pa) / (pb - pa);
  x[0] = ((double)u0 + (a == 0 ? t : 0.0)) * s[0] - o[0];
  x[1] = ((double)u1 + (a == 1 ? t : 0.0)) * s[1] - o[1];
  x[2] = ((double)u2 + (a == 2 ? t : 0.0)) * s[2] - o[2];
}

struct D3 {
  double x, y, z;
};

__device__ inline D3 sub3(const D3& a, const D3& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline D3 cross3(const D3& a, const D3& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// p at (z, y, x), 0 outside the array; the load is always issued (at a
// clamped address) so that several of them are in flight together.
__device__ inline double pld(const float* p, const int* d, int z, int y, int x) {
  const bool ok = (unsigned)z < (unsigned)d[0] && (unsigned)y < (unsigned)d[1] && (unsigned)x < (unsigned)d[2];
  const int zc = min(max(z, 0), d[0] - 1), yc = min(max(y, 0), d[1] - 1), xc = min(max(x, 0), d[2] - 1);
  const float v = p[((size_t)zc * d[1] + yc) * (size_t)d[2] + xc];
  return ok ? (double)v : 0.0;
}

// v[k] for a register array indexed by a run-time k in [0, 8) (selects, no scratch).
__device__ inline double sel8(const double* v, int k) {
  const double a = (k & 1) ? v[1] : v[0], b = (k & 1) ? v[3] : v[2];
  const double c = (k & 1) ? v[5] : v[4], e = (k & 1) ? v[7] : v[6];
  const double ab = (k & 2) ? b : a, ce = (k & 2) ? e : c;
  return (k & 4) ? ce : ab;
}

// Position (relative to o) of the vertex on cube edge e of the cube with min
// corner (c0, c1, c2) and corner values pc.
__device__ inline D3 cube_vertex(const double* pc, int e, int c0, int c1, int c2, const double* s, const double* o) {
  const int ea = MC_EDGE_AXIS[e], k0 = MC_EDGE_C0[e];
  const int k1 = k0 | (4 >> ea);
  const double p0 = sel8(pc, k0), p1 = sel8(pc, k1);
  const double tt = (0.5 - p0) / (p1 - p0);
  const int w0 = c0 + ((k0 >> 2) & 1), w1 = c1 + ((k0 >> 1) & 1), w2 = c2 + (k0 & 1);
  return {((double)w0 + (ea == 0 ? tt : 0.0)) * s[0] - o[0], ((double)w1 + (ea == 1 ? tt : 0.0)) * s[1] - o[1],
          ((double)w2 + (ea == 2 ? tt : 0.0)) * s[2] - o[2]};
}

// dL/dx of the vertex on edge (u, a) from the area and volume terms.
__device__ inline void vertex_grad_mesh(const float* p, const int* d, const double* s, const double* o, int u0, int u1,
                                        int u2, int a, double g_area, double g_vol_signed, double* gx) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int ob = q >> 1, oc = q & 1;
    // min corner of the cube: the edge's two other axes step back by ob and oc
    const int c0 = u0 - (a != 0 ? ob : 0);
    const int c1 = u1 - (a == 0 ? ob : (a == 1 ? 0 : oc));
    const int c2 = u2 - (a == 2 ? 0 : oc);
    const int le = 4 * a + 2 * ob + oc;  // the edge's number inside this cube
    double pc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) pc[k] = pld(p, d, c0 + ((k >> 2) & 1), c1 + ((k >> 1) & 1), c2 + (k & 1));
    int cas = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) cas |= (int)(pc[k] > 0.5) << k;
    const int nt = MC_NTRI[cas];
    for (int t = 0; t < nt; ++t) {
      const int e0 = MC_TRI[cas][t][0], e1 = MC_TRI[cas][t][1], e2 = MC_TRI[cas][t][2];
      if (e0 != le && e1 != le && e2 != le) continue;
      const D3 P0 = cube_vertex(pc, e0, c0, c1, c2, s, o);
      const D3 P1 = cube_vertex(pc, e1, c0, c1, c2, s, o);
      const D3 P2 = cube_vertex(pc, e2, c0, c1, c2, s, o);
      // B, C: the next two vertices after this one in the triangle's order
      const D3 B = e0 == le ? P1 : (e1 == le ? P2 : P0);
      const D3 C = e0 == le ? P2 : (e1 == le ? P0 : P1);
      const D3 n = cross3(sub3(P1, P0), sub3(P2, P0));
      const double len = sqrt(n.x * n.x + n.y * n.y + n.z * n.z);
      if (len > 0.0) {
        const D3 nh = {n.x / len, n.y / len, n.z / len};
        const D3 r = cross3(nh, sub3(C, B));
        gx[0] += g_area * 0.5 * r.x;
        gx[1] += g_area * 0.5 * r.y;
        gx[2] += g_area * 0.5 * r.z;
      }
      const D3 bc = cross3(B, C);
      gx[0] += g_vol_signed * bc.x / 6.0;
      gx[1] += g_vol_signed * bc.y / 6.0;
      gx[2] += g_vol_signed * bc.z / 6.0;
    }
  }
}

constexpr int kRowsPerWave = 8;
constexpr int kRowsPerBlock = 4 * kRowsPerWave;

// Last ROI whose first padded row (voxel row) is <= row.
__device__ inline int soft_roi_of_row(const SoftBwdRoi* r, int n, long long row) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (r[mid].row_begin <= row)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ inline int soft_roi_of_vrow(const SoftBwdRoi* r, int n, long long vrow) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (r[mid].vrow_begin <= vrow)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// A voxel row (z, y) of a ROI: its first element and whether it lies inside
// the array (an outside row reads row 0 and reports 0: the zero pad).
struct RowPtr {
  const float* ptr;
  bool ok;
};

__device__ inline RowPtr row_ptr(const float* p, const int* d, int z, int y) {
  const bool ok = (unsigned)z < (unsigned)d[0] && (unsigned)y < (unsigned)d[1];
  return {p + ((size_t)(ok ? z : 0) * d[1] + (ok ? y : 0)) * (size_t)d[2], ok};
}

// Element x in [0, d2) of a row, 0 if the row is outside the array (its
// pointer then addresses row 0, so the load is always in range).
__device__ inline float row_in(const RowPtr& r, int x) {
  const float v = r.ptr[x];
  return r.ok ? v : 0.0f;
}

// Element x of a row, 0 outside; the load is always issued at a clamped address.
__device__ inline float row_ld(const RowPtr& r, int x, int d2) {
  const float v = r.ptr[min(max(x, 0), d2 - 1)];
  return r.ok && (unsigned)x < (unsigned)d2 ? v : 0.0f;
}

__device__ inline int soft_roi_of_slot(const SoftBwdRoi* r, int n, long long slot) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (r[mid].field_begin <= slot)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Bit a set iff the edge (u, u + e_a) crosses the 0.5 level; A, Z, Y are the
// rows (u0, u1), (u0 + 1, u1), (u0, u1 + 1).
__device__ inline unsigned crossing_bits(const RowPtr& A, const RowPtr& Z, const RowPtr& Y, int u2, int d2) {
  const float va = row_ld(A, u2, d2), vz = row_ld(Z, u2, d2), vy = row_ld(Y, u2, d2), vx = row_ld(A, u2 + 1, d2);
  const bool c = va > 0.5f;
  return (unsigned)((vz > 0.5f) != c) | ((unsigned)((vy > 0.5f) != c) << 1) | ((unsigned)((vx > 0.5f) != c) << 2);
}

// Walks consecutive padded rows (u0, u1) of the ROI table: one ROI lookup
// and one division per wave, then increments.
struct PaddedRowWalk {
  const SoftBwdRoi* rois;
  int n, r;
  const SoftBwdRoi* R;
  int u0, u1;

  __device__ void start(const SoftBwdRoi* rs, int nr, long long row) {
    rois = rs;
    n = nr;
    r = soft_roi_of_row(rs, nr, row);
    R = rs + r;
    const long long lr = row - R->row_begin;
    u0 = (int)(lr / (R->d[1] + 1)) - 1;
    u1 = (int)(lr % (R->d[1] + 1)) - 1;
  }
  __device__ void next() {
    if (++u1 == R->d[1]) {
      u1 = -1;
      if (++u0 == R->d[0] && r + 1 < n) {
        R = rois + ++r;
        u0 = -1;
      }
    }
  }
};

// Crossing bits of the cubes u2 = x1 - 1 and x1 + 63 of a padded row (two
// chunks of 64 cubes per step, all eight loads issued together); 0 past the row.
__device__ inline void row_bits2(const RowPtr& A, const RowPtr& Z, const RowPtr& Y, int x1, int d2, unsigned& b0,
                                 unsigned& b1) {
  b0 = crossing_bits(A, Z, Y, x1 - 1, d2);
  b1 = crossing_bits(A, Z, Y, x1 + 63, d2);
  b0 = x1 <= d2 ? b0 : 0u;
  b1 = x1 + 64 <= d2 ? b1 : 0u;
}

// Crossing bits of every cube of a padded row with at most 64 * NC cubes:
// chunk c (cubes u2 = 64c - 1 + lane) in bits 3c .. 3c + 2 of the result.
// Chunks past the row end are skipped (a uniform branch); the loads of the
// others are all issued before any is used.
template <int NC>
__device__ inline uint32_t row_bits_all(const RowPtr& A, const RowPtr& Z, const RowPtr& Y, int lane, int d2) {
  float va[NC], vz[NC], vy[NC], vx[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (64 * c > d2) break;
    const int x1 = min(64 * c + lane, d2);  // u2 + 1
    const int i0 = max(x1 - 1, 0), i1 = min(x1, d2 - 1);
    va[c] = A.ptr[i0];
    vz[c] = Z.ptr[i0];
    vy[c] = Y.ptr[i0];
    vx[c] = A.ptr[i1];
  }
  uint32_t out = 0u;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (64 * c > d2) break;
    const int x1 = 64 * c + lane;
    const bool lo_ok = x1 >= 1, hi_ok = x1 <= d2 - 1;  // voxels u2 and u2 + 1 inside the row
    const bool in = A.ok && lo_ok && va[c] > 0.5f;
    const bool iz = Z.ok && lo_ok && vz[c] > 0.5f;
    const bool iy = Y.ok && lo_ok && vy[c] > 0.5f;
    const bool ix = A.ok && hi_ok && vx[c] > 0.5f;
    const uint32_t b = (uint32_t)(iz != in) | ((uint32_t)(iy != in) << 1) | ((uint32_t)(ix != in) << 2);
    out |= (x1 <= d2 ? b : 0u) << (3 * c);
  }
  return out;
}

// Cached crossing bits of a row (see row_bits_all), or kUncached for rows of
// more than 512 cubes, whose bits are recomputed chunk by chunk.
constexpr uint32_t kUncached = 0x80000000u;

__device__ inline uint32_t row_bits_cached(const RowPtr& A, const RowPtr& Z, const RowPtr& Y, int lane, int d2) {
  if (d2 + 1 <= 256) return row_bits_all<4>(A, Z, Y, lane, d2);
  if (d2 + 1 <= 512) return row_bits_all<8>(A, Z, Y, lane, d2);
  return kUncached;
}

__global__ __launch_bounds__(256) void k_soft_edges(SoftBwdBufs B) {
  __shared__ int cnt[kRowsPerBlock];
  __shared__ long long pre[kRowsPerBlock];
  __shared__ long long base_sh;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const long long row0 = (long long)blockIdx.x * kRowsPerBlock;
  const long long wrow0 = row0 + wid * kRowsPerWave;
  // pass 1: crossing edges per row; the bits of short rows stay in registers
  uint32_t cache[kRowsPerWave];
  {
    PaddedRowWalk W;
    if (wrow0 < B.n_rows) W.start(B.rois, B.n_rois, wrow0);
#pragma unroll
    for (int k = 0; k < kRowsPerWave; ++k) {
      const long long row = wrow0 + k;
      int c = 0;
      cache[k] = 0u;
      if (row < B.n_rows) {
        const SoftBwdRoi* R = W.R;
        const int d2 = R->d[2];
        const RowPtr A = row_ptr(R->p, R->d, W.u0, W.u1), Z = row_ptr(R->p, R->d, W.u0 + 1, W.u1),
                     Y = row_ptr(R->p, R->d, W.u0, W.u1 + 1);
        cache[k] = row_bits_cached(A, Z, Y, lane, d2);
        if (cache[k] != kUncached) {
          c = wave_sum(__popc(cache[k]));
        } else {
          for (int x0 = 0; x0 <= d2; x0 += 128) {
            unsigned b0, b1;
            row_bits2(A, Z, Y, x0 + lane, d2, b0, b1);
            c += __popc(b0) + __popc(b1);
          }
          c = wave_sum(c);
        }
        W.next();
      }
      if (lane == 0) cnt[wid * kRowsPerWave + k] = c;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long tot = 0;
    for (int i = 0; i < kRowsPerBlock; ++i) {
      pre[i] = tot;
      tot += cnt[i];
    }
    long long base = 0;
    if (tot > 0) base = (long long)atomicAdd((unsigned long long*)B.counters, (unsigned long long)tot);
    base_sh = base + tot <= B.cap ? base : -1;  // -1: no room (the input differs from the forward pass)
  }
  __syncthreads();
  const long long base = base_sh;
  if (base < 0 || wrow0 >= B.n_rows) return;
  // pass 2: write the rows' edges (field slots), in (row, u2, a) order
  PaddedRowWalk W;
  W.start(B.rois, B.n_rois, wrow0);
  const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
  for (int k = 0; k < kRowsPerWave; ++k) {
    const int li = wid * kRowsPerWave + k;
    const long long row = wrow0 + k;
    if (row >= B.n_rows) break;
    if (cnt[li] != 0) {
      const SoftBwdRoi* R = W.R;
      const int d2 = R->d[2];
      const RowPtr A = row_ptr(R->p, R->d, W.u0, W.u1), Z = row_ptr(R->p, R->d, W.u0 + 1, W.u1),
                   Y = row_ptr(R->p, R->d, W.u0, W.u1 + 1);
      long long off = base + pre[li];
      // slot of cube (u0, u1, -1) of this row: the row's local index times d2 + 1
      const long long slot0 = R->field_begin + 3ll * (row - R->row_begin) * (d2 + 1);
      for (int x0 = 0; x0 <= d2; x0 += 64) {
        const int x1 = x0 + lane;  // u2 + 1
        unsigned b;
        if (cache[k] != kUncached) {
          b = (cache[k] >> (3 * (x0 >> 6))) & 7u;
        } else {
          unsigned b1;
          row_bits2(A, Z, Y, x1, d2, b, b1);
        }
        const unsigned long long m0 = __ballot(b & 1u), m1 = __ballot(b & 2u), m2 = __ballot(b & 4u);
        long long slot = off + __popcll(m0 & below) + __popcll(m1 & below) + __popcll(m2 & below);
        for (int a = 0; a < 3; ++a)
          if ((b >> a) & 1u) B.edges[slot++] = (unsigned long long)(slot0 + 3ll * x1 + a);
        off += __popcll(m0) + __popcll(m1) + __popcll(m2);
      }
    }
    W.next();
  }
}

__global__ __launch_bounds__(256) void k_soft_vertex_grad(SoftBwdBufs B) {
  const long long n = min(B.counters[0], B.cap);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const long long slot = (long long)B.edges[i];
    // an entry no block wrote (only when the input has more crossing edges
    // than the forward pass: the call then fails) must not address memory
    if (slot < 0 || slot >= B.n_field) continue;
    const SoftBwdRoi* R = B.rois + soft_roi_of_slot(B.rois, B.n_rois, slot);
    const long long local = slot - R->field_begin;
    const int a = (int)(local % 3);
    const long long cube = local / 3;
    const int u2 = (int)(cube % (R->d[2] + 1)) - 1;
    const long long lr = cube / (R->d[2] + 1);
    const int u0 = (int)(lr / (R->d[1] + 1)) - 1, u1 = (int)(lr % (R->d[1] + 1)) - 1;
    double gx[3] = {0.0, 0.0, 0.0};
    vertex_grad_mesh(R->p, R->d, R->s, R->o, u0, u1, u2, a, R->g_area, R->g_vol_signed, gx);
    const long long id = 3ll * ((((long long)(u0 + 1)) * (R->d[1] + 2) + (u1 + 1)) * (long long)(R->d[2] + 2) +
                                (u2 + 1)) +
                         a;
    for (int f = 0; f < 4; ++f) {
      const double gd = R->gdiam[f];
      if (gd == 0.0) continue;
      const long long i_id = R->pair_ids[f][0], j_id = R->pair_ids[f][1];
      if (id != i_id && id != j_id) continue;
      const long long other = id == i_id ? j_id : i_id;
      const long long lin = other / 3;
      const int oa = (int)(other % 3);
      const int o2 = (int)(lin % (R->d[2] + 2)) - 1;
      const long long l2 = lin / (R->d[2] + 2);
      const int o1 = (int)(l2 % (R->d[1] + 2)) - 1;
      const int o0 = (int)(l2 / (R->d[1] + 2)) - 1;
      double xv[3], xo[3];
      vertex_pos(R->p, R->d, R->s, R->o, u0, u1, u2, a, xv);
      vertex_pos(R->p, R->d, R->s, R->o, o0, o1, o2, oa, xo);
      // dD/dx_v = (x_v - x_other) / D for either end point
      for (int c = 0; c < 3; ++c) gx[c] += gd * (xv[c] - xo[c]);
    }
    B.field[slot] = (float)(gx[a] * R->s[a]);
  }
}

// dL/dp of voxel w from its value vc and its six neighbours nv (indexed
// 2a + (neighbour is w + e_a)); slot_w is the field slot of edge (w, axis 0)
// and stride[a] the slot distance between the edges (w - e_a, a) and (w, a).
__device__ inline double voxel_grad(const float* __restrict__ field, long long slot_w, const long long* stride,
                                    float vc, const float* nv) {
  const bool in_w = vc > 0.5f;
  bool cross[6];
  bool any = false;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    cross[j] = (nv[j] > 0.5f) != in_w;
    any |= cross[j];
  }
  double g = 0.0;
  if (__ballot(any)) {
    // every lane loads all six slots (its own edge (w, 0) stands in where an
    // edge does not cross), so the loads issue together
    float q[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const int a = j >> 1;
      const long long sl = slot_w + a - ((j & 1) ? 0 : stride[a]);
      q[j] = field[cross[j] ? sl : slot_w];
    }
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      if (!cross[j]) continue;
      const bool up = j & 1;  // the neighbour is w + e_a (w is the edge's lower end)
      const double pu = up ? (double)vc : (double)nv[j], pb = up ? (double)nv[j] : (double)vc;
      const double den = pb - pu;
      g += (double)q[j] * (up ? (0.5 - pb) / (den * den) : -(0.5 - pu) / (den * den));
    }
  }
  return g;
}

// One wave per voxel row: up to 256 voxels (four per lane) per step, with all
// 28 loads of a step issued before any is used, so that a wave waits for
// memory once per 256 voxels.
__global__ __launch_bounds__(256) void k_soft_gather(SoftBwdBufs B) {
  constexpr int kV = 4;  // voxels per lane per step
  const int lane = threadIdx.x & 63;
  const long long vrow = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (vrow >= B.n_vrows) return;
  const SoftBwdRoi* R = B.rois + soft_roi_of_vrow(B.rois, B.n_rois, vrow);
  const int* d = R->d;
  const float* p = R->p;
  const int d2 = d[2];
  const long long lr = vrow - R->vrow_begin;
  const int w0 = (int)(lr / d[1]), w1 = (int)(lr % d[1]);
  // slot of edge ((w0, w1, -1), axis 0); voxel x adds 3 (x + 1)
  const long long slot_row = R->field_begin + 3ll * ((long long)(w0 + 1) * (d[1] + 1) + (w1 + 1)) * (d2 + 1);
  const long long stride[3] = {3ll * (d[1] + 1) * (d2 + 1), 3ll * (d2 + 1), 3};
  const RowPtr C = row_ptr(p, d, w0, w1), Zm = row_ptr(p, d, w0 - 1, w1), Zp = row_ptr(p, d, w0 + 1, w1),
               Ym = row_ptr(p, d, w0, w1 - 1), Yp = row_ptr(p, d, w0, w1 + 1);
  float* grow = R->grad + ((size_t)w0 * d[1] + w1) * (size_t)d2;
  for (int x0 = 0; x0 < d2; x0 += 64 * kV) {
    // lanes past the row end sit out (the wave's vote inside voxel_grad only
    // counts active lanes); addresses are the uniform row bases plus x
    float vc[kV], nv[kV][6];
#pragma unroll
    for (int h = 0; h < kV; ++h) {
      const int x = min(x0 + 64 * h + lane, d2 - 1);
      vc[h] = C.ptr[x];
      nv[h][0] = row_in(Zm, x);
      nv[h][1] = row_in(Zp, x);
      nv[h][2] = row_in(Ym, x);
      nv[h][3] = row_in(Yp, x);
      const float xm = C.ptr[max(x - 1, 0)], xp = C.ptr[min(x + 1, d2 - 1)];
      nv[h][4] = x > 0 ? xm : 0.0f;
      nv[h][5] = x < d2 - 1 ? xp : 0.0f;
    }
#pragma unroll
    for (int h = 0; h < kV; ++h) {
      const int x = x0 + 64 * h + lane;
      if (x < d2) grow[x] = (float)voxel_grad(B.field, slot_row + 3ll * (x + 1), stride, vc[h], nv[h]);
    }
  }
}

hipError_t launch_soft_backward(const SoftBwdBufs& B, hipStream_t st) {
  hipError_t e;
  if ((e = launch_fill_i64(B.counters, 0, 1, st))) return e;
  const long long nb = (B.n_rows + kRowsPerBlock - 1) / kRowsPerBlock;
  if (nb > 0) hipLaunchKernelGGL(k_soft_edges, dim3((unsigned)nb), dim3(256), 0, st, B);
  if ((e = hipGetLastError())) return e;
  long long g = (B.cap + 255) / 256;
  const long long gcap = (long long)B.cu_count * 16;
  if (g > gcap) g = gcap;
  if (g > 0) hipLaunchKernelGGL(k_soft_vertex_grad, dim3((unsigned)g), dim3(256), 0, st, B);
  if ((e = hipGetLastError())) return e;
  const long long nv = (B.n_vrows + 3) / 4;  // four voxel rows (waves) per workgroup
  if (nv > 0) hipLaunchKernelGGL(k_soft_gather, dim3((unsigned)nv), dim3(256), 0, st, B);
  return hipGetLastError();
}

}  // namespace s3d
