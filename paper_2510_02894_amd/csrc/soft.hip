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
//      computes (dL/dx_v)_a * s_a / (p_b - p_u)^2 into the edge's field slot;
//   3. k_soft_gather: for each voxel, the terms of its (at most six) incident
//      crossing edges, the field value times (0.5 - p_b) or -(0.5 - p_u), read
//      directly from their field slots, summed, and dL/dp written densely (0
//      away from the surface).  The division by (p_b - p_u)^2 is thus done once
//      per crossing edge, not once per end point over whole waves.
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
// corner (c0, c1, c2) and corner values pc.  Edge e = 4 axis + 2 o_b + o_c runs
// from corner k0 (bits dz dy dx) along its axis.
__device__ inline D3 cube_vertex(const double* pc, int e, int c0, int c1, int c2, const double* s, const double* o) {
  const int ea = e >> 2;
  const int k0 = ea == 0 ? (e & 3) : (ea == 1 ? 4 * ((e >> 1) & 1) + (e & 1) : 4 * ((e >> 1) & 1) + 2 * (e & 1));
  const int k1 = k0 | (4 >> ea);
  const double p0 = sel8(pc, k0), p1 = sel8(pc, k1);
  const double tt = (0.5 - p0) * rcp64(p1 - p0);
  const int w0 = c0 + ((k0 >> 2) & 1), w1 = c1 + ((k0 >> 1) & 1), w2 = c2 + (k0 & 1);
  return {((double)w0 + (ea == 0 ? tt : 0.0)) * s[0] - o[0], ((double)w1 + (ea == 1 ? tt : 0.0)) * s[1] - o[1],
          ((double)w2 + (ea == 2 ? tt : 0.0)) * s[2] - o[2]};
}

// dL/dx of the vertex on edge (u, a) from the area and volume terms; tri is
// the case table's edge triples and tmask[12 case + e] the set of the case's
// triangles that hold edge e (both in LDS).
__device__ inline void vertex_grad_mesh(const float* p, const int* d, const double* s, const double* o, int u0, int u1,
                                        int u2, int a, double g_area, double g_vol_signed, const uint8_t* tmask,
                                        const uint8_t* tri, double* gx) {
  // per-edge factors of the two terms (divisions hoisted out of the triangle loop)
  const double ga = 0.5 * g_area, gv = g_vol_signed / 6.0;
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
    // only the triangles that hold this vertex
    for (unsigned int m = tmask[cas * 12 + le]; m; m &= m - 1u) {
      const int t = __ffs(m) - 1;
      const uint8_t* tr = tri + (cas * MC_MAX_TRI + t) * 3;
      const int e0 = tr[0], e1 = tr[1], e2 = tr[2];
      const D3 P0 = cube_vertex(pc, e0, c0, c1, c2, s, o);
      const D3 P1 = cube_vertex(pc, e1, c0, c1, c2, s, o);
      const D3 P2 = cube_vertex(pc, e2, c0, c1, c2, s, o);
      // B, C: the next two vertices after this one in the triangle's order
      const D3 B = e0 == le ? P1 : (e1 == le ? P2 : P0);
      const D3 C = e0 == le ? P2 : (e1 == le ? P0 : P1);
      const D3 n = cross3(sub3(P1, P0), sub3(P2, P0));
      const double len = sqrt(n.x * n.x + n.y * n.y + n.z * n.z);
      if (len > 0.0) {
        const double il = rcp64(len);
        const D3 nh = {n.x * il, n.y * il, n.z * il};
        const D3 r = cross3(nh, sub3(C, B));
        gx[0] += ga * r.x;
        gx[1] += ga * r.y;
        gx[2] += ga * r.z;
      }
      const D3 bc = cross3(B, C);
      gx[0] += gv * bc.x;
      gx[1] += gv * bc.y;
      gx[2] += gv * bc.z;
    }
  }
}


// Last ROI whose first element of the given kind is <= x.
#define S3D_SOFT_ROI_SEARCH(name, member)                                   \
  __device__ inline int name(const SoftBwdRoi* r, int n, long long x) {     \
    int lo = 0, hi = n - 1;                                                  \
    while (lo < hi) {                                                        \
      const int mid = (lo + hi + 1) >> 1;                                    \
      if (r[mid].member <= x)                                                \
        lo = mid;                                                            \
      else                                                                   \
        hi = mid - 1;                                                        \
    }                                                                        \
    return lo;                                                               \
  }
S3D_SOFT_ROI_SEARCH(soft_roi_of_cblk, cblk_begin)
S3D_SOFT_ROI_SEARCH(soft_roi_of_vblk, vblk_begin)
#undef S3D_SOFT_ROI_SEARCH

// Pass 1.  A workgroup takes kCubeBlock consecutive cubes (flat index l over
// [-1, d-1]^3, the cube's edge-field index) of one ROI, 16 per thread; the
// crossing edges are counted, room is reserved with one atomic per workgroup
// and their field slots written in (thread, cube, axis) order.
__global__ __launch_bounds__(256) void k_soft_edges(SoftBwdBufs B) {
  constexpr int kPer = kCubeBlock / 256;
  __shared__ int s_scan[4];
  __shared__ long long base_sh;
  const int roi = B.blk_roi ? B.blk_roi[blockIdx.x] : soft_roi_of_cblk(B.rois, B.n_rois, blockIdx.x);
  const SoftBwdRoi* R = B.rois + roi;
  const int* d = R->d;
  const float* p = R->p;
  const unsigned int l0 = (unsigned int)(blockIdx.x - R->cblk_begin) * kCubeBlock + threadIdx.x;
  const unsigned int plane = (unsigned int)d[1] * d[2];
  unsigned long long bits = 0ull;  // 3 bits per cube k
#pragma unroll
  for (int h = 0; h < kPer; h += 8) {
    float v[8][4];
    bool ok[8][4];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const unsigned int l = l0 + 256u * (h + k);
      const unsigned int c0 = fdiv(l, R->m_cplane, R->sh_cplane);
      const unsigned int r = l - c0 * (unsigned int)((d[1] + 1) * (d[2] + 1));
      const unsigned int c1 = fdiv(r, R->m_c2, R->sh_c2);
      const int u0 = (int)c0 - 1, u1 = (int)c1 - 1, u2 = (int)(r - c1 * (unsigned int)(d[2] + 1)) - 1;
      const bool in_rng = l < R->n_cubes;
      const bool lo0 = u0 >= 0, lo1 = u1 >= 0, lo2 = u2 >= 0;
      // voxel index of u, with each coordinate clamped to 0 (the +axis
      // neighbours below step from it; a clamped axis means that neighbour
      // is the voxel at 0 on that axis)
      const unsigned int iv = in_rng ? ((unsigned int)max(u0, 0) * d[1] + max(u1, 0)) * d[2] + max(u2, 0) : 0u;
      ok[k][0] = in_rng && lo0 && lo1 && lo2;
      ok[k][1] = in_rng && u0 + 1 < d[0] && lo1 && lo2;
      ok[k][2] = in_rng && lo0 && u1 + 1 < d[1] && lo2;
      ok[k][3] = in_rng && lo0 && lo1 && u2 + 1 < d[2];
      // neighbours along +axis: +plane, +d2, +1 (clamped to iv when outside)
      v[k][0] = p[iv];
      v[k][1] = p[ok[k][1] ? iv + plane - (lo0 ? 0u : plane) : 0u];
      v[k][2] = p[ok[k][2] ? iv + (unsigned int)d[2] - (lo1 ? 0u : (unsigned int)d[2]) : 0u];
      v[k][3] = p[ok[k][3] ? iv + 1u - (lo2 ? 0u : 1u) : 0u];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const bool c = ok[k][0] && v[k][0] > 0.5f;
      const unsigned long long b = (unsigned long long)((ok[k][1] && v[k][1] > 0.5f) != c) |
                                   ((unsigned long long)((ok[k][2] && v[k][2] > 0.5f) != c) << 1) |
                                   ((unsigned long long)((ok[k][3] && v[k][3] > 0.5f) != c) << 2);
      bits |= (l0 + 256u * (h + k) < R->n_cubes ? b : 0ull) << (3 * (h + k));
    }
  }
  int total;
  const int off = block_excl_scan256(__popcll(bits), s_scan, total);
  if (threadIdx.x == 0) {
    long long base = 0;
    if (total > 0) base = (long long)atomicAdd((unsigned long long*)B.counters, (unsigned long long)total);
    base_sh = base + total <= B.cap ? base : -1;  // -1: no room (the input differs from the forward pass)
  }
  __syncthreads();
  const long long base = base_sh;
  if (base < 0) return;
  long long slot = base + off;
  while (bits) {
    const int i = __ffsll((long long)bits) - 1;
    bits &= bits - 1ull;
    const int k = i / 3, a = i - 3 * k;
    B.edges[slot++] = ((unsigned long long)roi << 40) | (3ull * (l0 + 256u * k) + (unsigned long long)a);
  }
}

__global__ __launch_bounds__(256, 3) void k_soft_vertex_grad(SoftBwdBufs B) {
  // the case table in LDS: its lookups depend on one another (case, then
  // triangle, then edge); per case and edge, the triangles that hold the edge
  __shared__ uint8_t s_tmask[256 * 12];
  __shared__ uint8_t s_tri[256 * MC_MAX_TRI * 3];
  for (int i = threadIdx.x; i < 256 * MC_MAX_TRI * 3; i += blockDim.x) s_tri[i] = (&MC_TRI[0][0][0])[i];
  for (int i = threadIdx.x; i < 256 * 12; i += blockDim.x) {
    const int c = i / 12, e = i - 12 * c;
    unsigned int m = 0u;
    for (int t = 0; t < MC_NTRI[c]; ++t)
      if (MC_TRI[c][t][0] == e || MC_TRI[c][t][1] == e || MC_TRI[c][t][2] == e) m |= 1u << t;
    s_tmask[i] = (uint8_t)m;
  }
  __syncthreads();
  const long long n = min(B.counters[0], B.cap);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const unsigned long long entry = B.edges[i];
    const unsigned int roi = (unsigned int)(entry >> 40);
    const unsigned long long local = entry & ((1ull << 40) - 1ull);
    // an entry no block wrote (only when the input has more crossing edges
    // than the forward pass: the call then fails) must not address memory
    if (roi >= (unsigned int)B.n_rois) continue;
    const SoftBwdRoi* R = B.rois + roi;
    if (local >= 3ull * R->n_cubes) continue;
    const long long slot = R->field_begin + (long long)local;
    // local = 3 cube(u) + a with cube(u) < 2^31: 32-bit decoding
    const unsigned int l32 = (unsigned int)local;
    const unsigned int cube = l32 / 3u;
    const int a = (int)(l32 - 3u * cube);
    const unsigned int c0 = fdiv(cube, R->m_cplane, R->sh_cplane);
    const unsigned int r = cube - c0 * (unsigned int)((R->d[1] + 1) * (R->d[2] + 1));
    const unsigned int c1 = fdiv(r, R->m_c2, R->sh_c2);
    const int u0 = (int)c0 - 1, u1 = (int)c1 - 1, u2 = (int)(r - c1 * (unsigned int)(R->d[2] + 1)) - 1;
    double gx[3] = {0.0, 0.0, 0.0};
    vertex_grad_mesh(R->p, R->d, R->s, R->o, u0, u1, u2, a, R->g_area, R->g_vol_signed, s_tmask, s_tri, gx);
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
    const double pu = pval(R->p, R->d, u0, u1, u2);
    const double pb = pval(R->p, R->d, u0 + (a == 0), u1 + (a == 1), u2 + (a == 2));
    const double den = pb - pu;  // at least one float ulp at 0.5: a crossing edge straddles it
    B.field[slot] = (float)(gx[a] * R->s[a] / (den * den));
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
      // the field holds (dL/dx_v)_a s_a / (p_b - p_u)^2; times dt/dp_w (p_b - p_u)^2
      g += (double)q[j] * (up ? 0.5 - (double)nv[j] : -(0.5 - (double)nv[j]));
    }
  }
  return g;
}

// Pass 3.  kVoxPer voxels per thread, 256 apart (flat index over the ROI,
// kVoxBlock per workgroup, so each load instruction of a wave reads 64
// consecutive floats), all 7 loads of each issued together; the voxel's
// crossing edges read their values from the edge field and dL/dp is written
// densely.
__global__ __launch_bounds__(256) void k_soft_gather(SoftBwdBufs B) {
  const SoftBwdRoi* R =
      B.rois + (B.blk_roi ? B.blk_roi[B.n_cblocks + blockIdx.x] : soft_roi_of_vblk(B.rois, B.n_rois, blockIdx.x));
  const unsigned int l0 = (unsigned int)(blockIdx.x - R->vblk_begin) * kVoxBlock + threadIdx.x;
  if (l0 >= R->n_vox) return;
  const int* d = R->d;
  const float* p = R->p;
  const unsigned int plane = (unsigned int)d[1] * d[2];
  const long long stride[3] = {3ll * (d[1] + 1) * (d[2] + 1), 3ll * (d[2] + 1), 3};
  float vc[kVoxPer], nv[kVoxPer][6];
  long long slot[kVoxPer];
#pragma unroll
  for (int j = 0; j < kVoxPer; ++j) {
    // voxels past the ROI's end repeat its last voxel (loaded, not written)
    const unsigned int l = min(l0 + 256u * j, R->n_vox - 1u);
    const unsigned int w0 = fdiv(l, R->m_plane, R->sh_plane);
    const unsigned int r = l - w0 * plane;
    const unsigned int w1 = fdiv(r, R->m_d2, R->sh_d2);
    const unsigned int x = r - w1 * (unsigned int)d[2];
    const bool zm = w0 > 0, zp = w0 + 1 < (unsigned int)d[0], ym = w1 > 0, yp = w1 + 1 < (unsigned int)d[1];
    const bool xm = x > 0, xp = x + 1 < (unsigned int)d[2];
    vc[j] = p[l];
    nv[j][0] = p[zm ? l - plane : l];
    nv[j][1] = p[zp ? l + plane : l];
    nv[j][2] = p[ym ? l - d[2] : l];
    nv[j][3] = p[yp ? l + d[2] : l];
    nv[j][4] = p[xm ? l - 1 : l];
    nv[j][5] = p[xp ? l + 1 : l];
    nv[j][0] = zm ? nv[j][0] : 0.0f;
    nv[j][1] = zp ? nv[j][1] : 0.0f;
    nv[j][2] = ym ? nv[j][2] : 0.0f;
    nv[j][3] = yp ? nv[j][3] : 0.0f;
    nv[j][4] = xm ? nv[j][4] : 0.0f;
    nv[j][5] = xp ? nv[j][5] : 0.0f;
    // field slot of edge (w, axis 0): 3 * cube(w)
    slot[j] = R->field_begin + 3ll * (((long long)(w0 + 1) * (d[1] + 1) + (w1 + 1)) * (d[2] + 1) + (x + 1));
  }
#pragma unroll
  for (int j = 0; j < kVoxPer; ++j) {
    const float g = (float)voxel_grad(B.field, slot[j], stride, vc[j], nv[j]);
    if (l0 + 256u * j < R->n_vox) R->grad[l0 + 256u * j] = g;
  }
}

// The ROI of every workgroup of the edge and gather passes (one workgroup per
// ROI writes its two contiguous block ranges).
__global__ void k_soft_block_rois(SoftBwdBufs B) {
  int* blk_roi = B.blk_roi;
  const SoftBwdRoi& R = B.rois[blockIdx.x];
  const long long nc = ((long long)R.n_cubes + kCubeBlock - 1) / kCubeBlock;
  const long long nv = ((long long)R.n_vox + kVoxBlock - 1) / kVoxBlock;
  for (long long i = threadIdx.x; i < nc; i += blockDim.x) blk_roi[R.cblk_begin + i] = (int)blockIdx.x;
  for (long long i = threadIdx.x; i < nv; i += blockDim.x) blk_roi[B.n_cblocks + R.vblk_begin + i] = (int)blockIdx.x;
}

hipError_t launch_soft_backward(const SoftBwdBufs& B, hipStream_t st) {
  hipError_t e;
  if ((e = launch_fill_i64(B.counters, 0, 1, st))) return e;
  if (B.blk_roi) hipLaunchKernelGGL(k_soft_block_rois, dim3((unsigned)B.n_rois), dim3(256), 0, st, B);
  if (B.n_cblocks > 0) hipLaunchKernelGGL(k_soft_edges, dim3((unsigned)B.n_cblocks), dim3(256), 0, st, B);
  if ((e = hipGetLastError())) return e;
  long long g = (B.cap + 255) / 256;
  const long long gcap = (long long)B.cu_count * 16;
  if (g > gcap) g = gcap;
  if (g > 0) hipLaunchKernelGGL(k_soft_vertex_grad, dim3((unsigned)g), dim3(256), 0, st, B);
  if ((e = hipGetLastError())) return e;
  if (B.n_vblocks > 0) hipLaunchKernelGGL(k_soft_gather, dim3((unsigned)B.n_vblocks), dim3(256), 0, st, B);
  return hipGetLastError();
}

}  // namespace s3d
