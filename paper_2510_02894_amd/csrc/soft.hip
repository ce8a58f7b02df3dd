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
// One thread per voxel gathers everything it needs (gather form, no float
// atomics: deterministic); a vertex's gradient is evaluated by both end points
// of its edge.  Voxels on no crossing edge write 0.
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

__global__ __launch_bounds__(256) void k_soft_backward(const float* __restrict__ p, SoftBwdArgs A,
                                                       float* __restrict__ grad) {
  const long long N = (long long)A.d[0] * A.d[1] * A.d[2];
  for (long long w = (long long)blockIdx.x * blockDim.x + threadIdx.x; w < N;
       w += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(w % A.d[2]);
    const long long r = w / A.d[2];
    const int y = (int)(r % A.d[1]);
    const int z = (int)(r / A.d[1]);
    const bool in_w = p[w] > 0.5f;
    double g = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int dir = -1; dir <= 1; dir += 2) {
        const int nz = z + (a == 0 ? dir : 0), ny = y + (a == 1 ? dir : 0), nx = x + (a == 2 ? dir : 0);
        if (pin(p, A.d, nz, ny, nx) == in_w) continue;
        // edge from u (lower end) along axis a
        const int u0 = dir > 0 ? z : nz, u1 = dir > 0 ? y : ny, u2 = dir > 0 ? x : nx;
        const double pu = pval(p, A.d, u0, u1, u2);
        const double pb = pval(p, A.d, u0 + (a == 0), u1 + (a == 1), u2 + (a == 2));
        const double den = pb - pu;
        const double dt = dir > 0 ? (0.5 - pb) / (den * den) : -(0.5 - pu) / (den * den);
        double gx[3] = {0.0, 0.0, 0.0};
        vertex_grad_mesh(p, A.d, A.s, A.o, u0, u1, u2, a, A.gout[1], A.g_vol_signed, gx);
        const unsigned long long id = 3ull * ((((unsigned long long)(u0 + 1)) * (A.d[1] + 2) + (u1 + 1)) *
                                                  (unsigned long long)(A.d[2] + 2) +
                                              (u2 + 1)) +
                                      a;
        for (int f = 0; f < 4; ++f) {
          if (!(A.D[f] > 0.0)) continue;
          const long long i_id = A.pair_ids[f][0], j_id = A.pair_ids[f][1];
          if ((long long)id != i_id && (long long)id != j_id) continue;
          const long long other = (long long)id == i_id ? j_id : i_id;
          // decode the partner's edge and position
          const long long lin = other / 3;
          const int oa = (int)(other % 3);
          const int o2 = (int)(lin % (A.d[2] + 2)) - 1;
          const long long l2 = lin / (A.d[2] + 2);
          const int o1 = (int)(l2 % (A.d[1] + 2)) - 1;
          const int o0 = (int)(l2 / (A.d[1] + 2)) - 1;
          double xv[3], xo[3];
          vertex_pos(p, A.d, A.s, A.o, u0, u1, u2, a, xv);
          vertex_pos(p, A.d, A.s, A.o, o0, o1, o2, oa, xo);
          // dD/dx_v = (x_v - x_other) / D for either end point
          for (int q = 0; q < 3; ++q) gx[q] += A.gout[2 + f] * (xv[q] - xo[q]) / A.D[f];
        }
        g += gx[a] * A.s[a] * dt;
      }
    grad[w] = (float)g;
  }
}

hipError_t launch_soft_backward(const float* p, const SoftBwdArgs& A, float* grad, int cu_count, hipStream_t st) {
  const long long N = (long long)A.d[0] * A.d[1] * A.d[2];
  long long g = (N + 255) / 256;
  const long long cap = (long long)cu_count * 32;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_soft_backward, dim3((unsigned)g), dim3(256), 0, st, p, A, grad);
  return hipGetLastError();
}

}  // namespace s3d
