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
//      edges in (u2, a) order; a workgroup reserves room for its rows with one
//      atomic and records each row's first entry and count;
//   2. k_soft_vertex_grad: one thread per crossing edge (the surface is sparse,
//      so a thread per voxel would leave most lanes idle around the FP64 work)
//      computes (dL/dx_v)_a * s_a;
//   3. k_soft_gather: one wave per voxel row sums, for each voxel, the terms of
//      its (at most six) incident crossing edges, found by binary search in the
//      edge's row, and writes dL/dp densely (0 away from the surface).
// No float atomics: the result does not depend on scheduling.
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

__device__ inline bool pin(const float* p, const int* d, int z, int y, int x) {
  if (z < 0 || y < 0 || x < 0 || z >= d[0] || y >= d[1] || x >= d[2]) return false;
  return p[((size_t)z * d[1] + y) * (size_t)d[2] + x] > 0.5f;
}

__device__ inline void cross3(const double* a, const double* b, double* r) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
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

// dL/dx of the vertex on edge (u, a) from the area and volume terms.
__device__ inline void vertex_grad_mesh(const float* p, const int* d, const double* s, const double* o, int u0, int u1,
                                        int u2, int a, double g_area, double g_vol_signed, double* gx) {
  const int b_ax = a == 0 ? 1 : 0, c_ax = a == 2 ? 1 : 2;
  for (int ob = 0; ob < 2; ++ob)
    for (int oc = 0; oc < 2; ++oc) {
      int c[3] = {u0, u1, u2};  // cube min corner
      c[b_ax] -= ob;
      c[c_ax] -= oc;
      const int le = 4 * a + 2 * ob + oc;  // the edge's number inside this cube
      double pc[8];
      int cas = 0;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int z = c[0] + ((k >> 2) & 1), y = c[1] + ((k >> 1) & 1), x = c[2] + (k & 1);
        pc[k] = pval(p, d, z, y, x);
        cas |= (int)pin(p, d, z, y, x) << k;
      }
      const int nt = MC_NTRI[cas];
      for (int t = 0; t < nt; ++t) {
        int k = -1;
        for (int v = 0; v < 3; ++v)
          if (MC_TRI[cas][t][v] == le) k = v;
        if (k < 0) continue;
        double P[3][3];
        for (int v = 0; v < 3; ++v) {
          const int e = MC_TRI[cas][t][v];
          const int ea = MC_EDGE_AXIS[e], c0 = MC_EDGE_C0[e];
          const int c1 = c0 | (4 >> ea);
          const double tt = (0.5 - pc[c0]) / (pc[c1] - pc[c0]);
          const int w0 = c[0] + ((c0 >> 2) & 1), w1 = c[1] + ((c0 >> 1) & 1), w2 = c[2] + (c0 & 1);
          P[v][0] = ((double)w0 + (ea == 0 ? tt : 0.0)) * s[0] - o[0];
          P[v][1] = ((double)w1 + (ea == 1 ? tt : 0.0)) * s[1] - o[1];
          P[v][2] = ((double)w2 + (ea == 2 ? tt : 0.0)) * s[2] - o[2];
        }
        const double* B = P[(k + 1) % 3];
        const double* C = P[(k + 2) % 3];
        double e1[3], e2[3], n[3];
        for (int q = 0; q < 3; ++q) {
          e1[q] = P[1][q] - P[0][q];
          e2[q] = P[2][q] - P[0][q];
        }
        cross3(e1, e2, n);
        const double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (len > 0.0) {
          const double nh[3] = {n[0] / len, n[1] / len, n[2] / len};
          const double cb[3] = {C[0] - B[0], C[1] - B[1], C[2] - B[2]};
          double r[3];
          cross3(nh, cb, r);
          for (int q = 0; q < 3; ++q) gx[q] += g_area * 0.5 * r[q];
        }
        double bc[3];
        cross3(B, C, bc);
        for (int q = 0; q < 3; ++q) gx[q] += g_vol_signed * bc[q] / 6.0;
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

// Bit a set iff the edge (u, u + e_a) crosses the 0.5 level.
__device__ inline unsigned crossing_bits(const float* p, const int* d, int u0, int u1, int u2) {
  const bool c = pin(p, d, u0, u1, u2);
  return (unsigned)(pin(p, d, u0 + 1, u1, u2) != c) | ((unsigned)(pin(p, d, u0, u1 + 1, u2) != c) << 1) |
         ((unsigned)(pin(p, d, u0, u1, u2 + 1) != c) << 2);
}

__global__ __launch_bounds__(256) void k_soft_edges(SoftBwdBufs B) {
  __shared__ int cnt[kRowsPerBlock];
  __shared__ long long pre[kRowsPerBlock];
  __shared__ long long base_sh;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const long long row0 = (long long)blockIdx.x * kRowsPerBlock;
  // pass 1: crossing edges per row
  for (int k = 0; k < kRowsPerWave; ++k) {
    const int li = wid * kRowsPerWave + k;
    const long long row = row0 + li;
    int c = 0;
    if (row < B.n_rows) {
      const SoftBwdRoi* R = B.rois + soft_roi_of_row(B.rois, B.n_rois, row);
      const long long lr = row - R->row_begin;
      const int u0 = (int)(lr / (R->d[1] + 1)) - 1, u1 = (int)(lr % (R->d[1] + 1)) - 1;
      for (int x0 = 0; x0 <= R->d[2]; x0 += 64) {
        const unsigned b = x0 + lane <= R->d[2] ? crossing_bits(R->p, R->d, u0, u1, x0 + lane - 1) : 0u;
        c += __popcll(__ballot(b & 1u)) + __popcll(__ballot(b & 2u)) + __popcll(__ballot(b & 4u));
      }
    }
    if (lane == 0) cnt[li] = c;
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
  if (threadIdx.x < kRowsPerBlock && row0 + threadIdx.x < B.n_rows) {
    B.row_base[row0 + threadIdx.x] = base >= 0 ? base + pre[threadIdx.x] : 0;
    B.row_cnt[row0 + threadIdx.x] = base >= 0 ? cnt[threadIdx.x] : 0;
  }
  if (base < 0) return;
  // pass 2: write the rows' edges, sorted by (u2, a)
  for (int k = 0; k < kRowsPerWave; ++k) {
    const int li = wid * kRowsPerWave + k;
    const long long row = row0 + li;
    if (row >= B.n_rows || cnt[li] == 0) continue;
    const SoftBwdRoi* R = B.rois + soft_roi_of_row(B.rois, B.n_rois, row);
    const long long lr = row - R->row_begin;
    const int u0 = (int)(lr / (R->d[1] + 1)) - 1, u1 = (int)(lr % (R->d[1] + 1)) - 1;
    long long off = base + pre[li];
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int x0 = 0; x0 <= R->d[2]; x0 += 64) {
      const int x1 = x0 + lane;  // u2 + 1
      const unsigned b = x1 <= R->d[2] ? crossing_bits(R->p, R->d, u0, u1, x1 - 1) : 0u;
      const unsigned long long m0 = __ballot(b & 1u), m1 = __ballot(b & 2u), m2 = __ballot(b & 4u);
      long long slot = off + __popcll(m0 & below) + __popcll(m1 & below) + __popcll(m2 & below);
      for (int a = 0; a < 3; ++a)
        if ((b >> a) & 1u) B.edges[slot++] = ((unsigned long long)row << 17) | (unsigned long long)(x1 * 3 + a);
      off += __popcll(m0) + __popcll(m1) + __popcll(m2);
    }
  }
}

__global__ __launch_bounds__(256) void k_soft_vertex_grad(SoftBwdBufs B) {
  const long long n = min(B.counters[0], B.cap);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const unsigned long long e = B.edges[i];
    const long long row = (long long)(e >> 17);
    const int key = (int)(e & 0x1FFFFull);
    const int a = key % 3, u2 = key / 3 - 1;
    const SoftBwdRoi* R = B.rois + soft_roi_of_row(B.rois, B.n_rois, row);
    const long long lr = row - R->row_begin;
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
    B.q[i] = gx[a] * R->s[a];
  }
}

// q of edge key (u2 + 1) * 3 + a of padded row `row` (0 if it is not listed).
__device__ inline double edge_q(const SoftBwdBufs& B, long long row, int key) {
  long long lo = B.row_base[row], hi = lo + B.row_cnt[row] - 1;
  while (lo <= hi) {
    const long long mid = (lo + hi) >> 1;
    const int k = (int)(B.edges[mid] & 0x1FFFFull);
    if (k == key) return B.q[mid];
    if (k < key)
      lo = mid + 1;
    else
      hi = mid - 1;
  }
  return 0.0;
}

__global__ __launch_bounds__(256) void k_soft_gather(SoftBwdBufs B) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = 0; k < kRowsPerWave; ++k) {
    const long long vrow = (long long)blockIdx.x * kRowsPerBlock + wid * kRowsPerWave + k;
    if (vrow >= B.n_vrows) break;
    const SoftBwdRoi* R = B.rois + soft_roi_of_vrow(B.rois, B.n_rois, vrow);
    const int* d = R->d;
    const float* p = R->p;
    const long long lr = vrow - R->vrow_begin;
    const int w0 = (int)(lr / d[1]), w1 = (int)(lr % d[1]);
    // padded row of the cube row (w0, w1); (w0, w1 - 1) is the one before it
    // and (w0 - 1, w1) the one d1 + 1 before it
    const long long rw = R->row_begin + (long long)(w0 + 1) * (d[1] + 1) + (w1 + 1);
    const size_t rbase = ((size_t)w0 * d[1] + w1) * (size_t)d[2];
    for (int x = lane; x < d[2]; x += 64) {
      const bool in_w = p[rbase + x] > 0.5f;
      double g = 0.0;
      for (int a = 0; a < 3; ++a)
        for (int dir = -1; dir <= 1; dir += 2) {
          const int nz = w0 + (a == 0 ? dir : 0), ny = w1 + (a == 1 ? dir : 0), nx = x + (a == 2 ? dir : 0);
          if (pin(p, d, nz, ny, nx) == in_w) continue;
          // the edge (u, u + e_a) with u = w (dir > 0) or w - e_a (dir < 0)
          const int u0 = dir > 0 ? w0 : nz, u1 = dir > 0 ? w1 : ny, u2 = dir > 0 ? x : nx;
          const long long row = dir > 0 || a == 2 ? rw : (a == 0 ? rw - (d[1] + 1) : rw - 1);
          const double q = edge_q(B, row, (u2 + 1) * 3 + a);
          const double pu = pval(p, d, u0, u1, u2);
          const double pb = pval(p, d, u0 + (a == 0), u1 + (a == 1), u2 + (a == 2));
          const double den = pb - pu;
          g += q * (dir > 0 ? (0.5 - pb) / (den * den) : -(0.5 - pu) / (den * den));
        }
      R->grad[rbase + x] = (float)g;
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
  const long long nv = (B.n_vrows + kRowsPerBlock - 1) / kRowsPerBlock;
  if (nv > 0) hipLaunchKernelGGL(k_soft_gather, dim3((unsigned)nv), dim3(256), 0, st, B);
  return hipGetLastError();
}

}  // namespace s3d
