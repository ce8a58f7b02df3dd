// mesh.hip -- the marching-cubes mesh pass (paper Sec. 2, "Marching cubes
// fused parallel kernels"): cube classification, vertex counting and
// emission, surface area and signed volume.
//
// A workgroup handles a brick: 256 row-groups (32 consecutive cubes along
// axis 2 of one cube row) times up to kTZ cube planes.  It first stages every
// voxel row-group the brick touches in LDS as 32-bit masks (all loads issued
// at once; each mask byte or float becomes one bit once), then each thread
// classifies its 32 cubes of every plane pair from LDS: crossing edges and
// active cubes come from bitwise operations on eight 32-bit corner masks, and
// only active cubes (a few percent) touch the case tables.
//
// Area and volume (binary masks): vertices sit at edge midpoints, so each
// case's area is a fixed number for the call's spacing and its volume term is
// an integer in units of s0*s1*s2/48 (see gen_mc_table.py).  The binary pass
// therefore accumulates the volume exactly in int64 and the area as FP64
// sums in a fixed order.  Soft masks evaluate every triangle in FP64.
//
// Inside-voxel moments (the principal-axis members of the Shape class, asked
// for per call): every voxel is the far corner (1, 1, 1) of exactly one cube,
// so the thread that owns that cube counts it, from the voxel-row word it
// already holds.  A word's count, sum of bit positions and sum of squared bit
// positions come from popcounts of the word under fixed bit patterns; the
// thread, brick and ROI sums are integers, so the second moments are exact
// and independent of the order of the work.
#include <hip/hip_runtime.h>

#include <algorithm>

#define MC_TABLE_QUAL __constant__ const
#include "mc_table.h"
#include "s3d_device.h"
#include "s3d_launch.h"

namespace s3d {

// ---------------------------------------------------------------------------
// Voxel bytes to inside bits, four at a time.

__device__ inline uint32_t nz4(uint32_t w) {
  // high bit of each byte set iff the byte is nonzero, then gathered to bits 0..3
  const uint32_t t = (((w & 0x7f7f7f7fu) + 0x7f7f7f7fu) | w) & 0x80808080u;
  return (t * 0x00204081u) >> 28;
}

// Bits 0..3 set for the bytes of w equal to the ROI's label (label != 0), or
// for its nonzero bytes (label == 0).
__device__ inline uint32_t in4(uint32_t w, uint32_t label4) {
  return label4 ? (~nz4(w ^ label4) & 0xfu) : nz4(w);
}

// Slots per chunk of a brick's dense enumeration of active cubes or crossing
// edges (8 per thread).
constexpr int kMeshItems = 2048;
static_assert(kMeshItems == 8 * kBrickThreads, "the slot scan gives each thread 8 slots");

// Position of the r-th set bit (r = 0 for the lowest) of w; r < popc(w).
__device__ inline int nth_set_bit(uint32_t w, int r) {
  int pos = 0;
#pragma unroll
  for (int h = 16; h >= 1; h >>= 1) {
    const int c = __popc(w & ((1u << h) - 1u));
    const bool up = r >= c;
    r = up ? r - c : r;
    w = up ? w >> h : w;
    pos = up ? pos + h : pos;
  }
  return pos;
}

// Inclusive max-scan of s[0, n) by the workgroup, 8 consecutive slots per
// thread (slots >= n read as 0).  s_mx holds 4 words.  Contains barriers.
__device__ inline void block_max_scan(uint32_t* s, int n, uint32_t* s_mx) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int b = 8 * tid;
  const uint4 q0 = *(const uint4*)(s + b), q1 = *(const uint4*)(s + b + 4);
  const uint32_t in[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
  uint32_t v[8], m = 0u;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    m = max(m, b + j < n ? in[j] : 0u);
    v[j] = m;
  }
  uint32_t x = m;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x = max(x, y);
  }
  const uint32_t prev = __shfl_up(x, 1, 64);
  if (lane == 63) s_mx[wid] = x;
  __syncthreads();
  uint32_t pre = lane > 0 ? prev : 0u;
  for (int w = 0; w < wid; ++w) pre = max(pre, s_mx[w]);
  *(uint4*)(s + b) = make_uint4(max(pre, v[0]), max(pre, v[1]), max(pre, v[2]), max(pre, v[3]));
  *(uint4*)(s + b + 4) = make_uint4(max(pre, v[4]), max(pre, v[5]), max(pre, v[6]), max(pre, v[7]));
  __syncthreads();
}

// Dense enumeration of the set bits of the brick's per-thread words: thread t
// holds NW words (their bit counts are passed, one per byte of `counts`), item
// numbers run over threads, then words, then bits, and `off` is the thread's
// first item.  For the chunk of items [c0, c0 + n), each
// nonempty word writes a marker at the slot where it begins (slot 0 for a word
// that began in an earlier chunk), (slot << 21) | (bits before the chunk << 16)
// | (t << 8) | word; the max-scan then leaves in every slot i the marker of the
// word that holds item c0 + i, which is that word's
// (i - (marker >> 21) + ((marker >> 16) & 31))-th set bit.  Every lane does
// the same amount of work however the bits fall among the threads.
template <int NW>
__device__ inline void mark_words(const uint32_t* counts, int off, int c0, int n, uint32_t* s, uint32_t* s_mx) {
  static_assert(NW <= 256, "the word index takes 8 bits");
  for (int i = threadIdx.x; i < n; i += kBrickThreads) s[i] = 0u;
  // The counts pass through an empty asm statement so that the compiler does
  // not hoist the NW word offsets out of the caller's chunk loop, which would
  // hold NW more registers through the whole kernel.
  uint32_t cc[(NW + 3) / 4];
#pragma unroll
  for (int q = 0; q < (NW + 3) / 4; ++q) {
    cc[q] = counts[q];
    asm volatile("" : "+v"(cc[q]));
  }
  __syncthreads();
  int o = off - c0;  // first item of word j, relative to the chunk
#pragma unroll
  for (int j = 0; j < NW; ++j) {
    const int c = (int)((cc[j >> 2] >> (8 * (j & 3))) & 0xffu);
    if (c > 0 && o + c > 0 && o < n) {
      const int ls = max(o, 0);
      s[ls] = ((uint32_t)ls << 21) | ((uint32_t)(ls - o) << 16) | ((uint32_t)threadIdx.x << 8) | (uint32_t)j;
    }
    o += c;
  }
  __syncthreads();
  block_max_scan(s, n, s_mx);
}

__device__ inline int marker_rank(uint32_t mk, int i) { return i - (int)(mk >> 21) + (int)((mk >> 16) & 31u); }

// v[k] of an 8-entry register array for a run-time k (selects, no scratch).
__device__ inline double sel8d(const double* v, int k) {
  const double a = (k & 1) ? v[1] : v[0], b = (k & 1) ? v[3] : v[2];
  const double c = (k & 1) ? v[5] : v[4], e = (k & 1) ? v[7] : v[6];
  const double ab = (k & 2) ? b : a, ce = (k & 2) ? e : c;
  return (k & 4) ? ce : ab;
}

__device__ inline double soft_value(const Roi& R, int z, int y, int x) {
  if (z < 0 || y < 0 || x < 0 || z >= R.d[0] || y >= R.d[1] || x >= R.d[2]) return 0.0;
  return (double)((const float*)R.vol)[(size_t)z * (size_t)R.stride0 + (size_t)y * (size_t)R.stride1 + (size_t)x];
}

// A brick is kBrickThreads consecutive row-groups (rg = cube row * G + group)
// times up to R.tz (at most kTZ) cube planes.  Its workgroup first loads, as bit masks, every
// voxel row-group it needs into LDS: planes pz0-1 .. pz1-1 and row-groups
// rg0-1 .. rg0+kBrickThreads+G-1 (the row after each cube row, and the word
// before the first group for the x-1 voxel).  All these loads are issued at
// once, each voxel row-group is converted once, and the cube classification
// then reads LDS only.
struct Tile {
  int rg0;       // first row-group of the brick
  int pz0, pz1;  // cube planes [pz0, pz1), pz = z + 1
  int np;        // voxel planes held: pz1 - pz0 + 1
  int nw;        // words per plane: kBrickThreads + 1 + G
};

__device__ inline Tile tile_of(const Roi& R, long long local_brick) {
  Tile T;
  const int bx = (int)(local_brick / R.nzc), zc = (int)(local_brick % R.nzc);
  T.rg0 = bx * kBrickThreads;
  T.pz0 = zc * R.tz;
  T.pz1 = min(T.pz0 + R.tz, R.d[0] + 1);
  T.np = T.pz1 - T.pz0 + 1;
  T.nw = kBrickThreads + 1 + R.G;
  return T;
}

// Voxel row-group vrg of voxel plane p of the tile: the address of its first
// voxel and the number of its 32 voxels that lie inside the array (0 when the
// row-group lies outside it; then the address is not used).
template <int DT>
__device__ inline const char* row_span(const Roi& R, const Tile& T, int p, int vrg, int& nvox) {
  nvox = 0;
  if (vrg < 0) return nullptr;
  const int ry = (int)fdiv((unsigned int)vrg, R.mG, R.shG);
  const int z = T.pz0 - 1 + p, y = ry - 1, x0 = 32 * (vrg - ry * R.G);
  if (z < 0 || z >= R.d[0] || y < 0 || y >= R.d[1] || x0 >= R.d[2]) return nullptr;
  nvox = min(32, R.d[2] - x0);
  const size_t off = (size_t)z * (size_t)R.stride0 + (size_t)y * (size_t)R.stride1 + (size_t)x0;
  return (const char*)R.vol + off * (DT == 0 ? 1 : 4);
}

// Stages the tile's voxel row-groups in LDS.  Each thread issues the loads of
// several row-groups before converting any of them, so a workgroup keeps its
// whole tile in flight instead of one row-group per thread at a time.  A full
// row-group at a 16-byte aligned address is read with 16-byte loads; any other
// (rows of packed ROIs start anywhere, row ends) with loads of the aligned
// dwords (uint8) or floats that hold its voxels inside the array, and never
// past them, since an aligned dword holding a valid byte lies on a mapped page.
template <int DT>
__device__ inline void load_tile(const Roi& R, const Tile& T, uint32_t* s_bits) {
  const int n = T.np * T.nw;
  if (DT == 0) {
    constexpr int kLoadBatch = 5;
    const uint32_t label4 = (uint32_t)(R.label & 0xff) * 0x01010101u;
    for (int base = threadIdx.x; base < n; base += kBrickThreads * kLoadBatch) {
      uint32_t d[kLoadBatch][9];
      int nv[kLoadBatch], sh[kLoadBatch];
#pragma unroll
      for (int u = 0; u < kLoadBatch; ++u) {
        const int idx = base + u * kBrickThreads;
        const char* ptr = nullptr;
        nv[u] = 0;
        sh[u] = 0;
#pragma unroll
        for (int j = 0; j < 9; ++j) d[u][j] = 0u;
        if (idx < n) {
          const int p = (int)fdiv((unsigned int)idx, R.mNW, R.shNW);
          ptr = row_span<DT>(R, T, p, T.rg0 - 1 + idx - p * T.nw, nv[u]);
        }
        if (nv[u] == 32 && (((uintptr_t)ptr) & 15u) == 0) {
          const uint4 a = *(const uint4*)ptr, b = *((const uint4*)ptr + 1);
          d[u][0] = a.x;
          d[u][1] = a.y;
          d[u][2] = a.z;
          d[u][3] = a.w;
          d[u][4] = b.x;
          d[u][5] = b.y;
          d[u][6] = b.z;
          d[u][7] = b.w;
        } else if (nv[u] > 0) {
          const uintptr_t a = (uintptr_t)ptr;
          const uint32_t* q = (const uint32_t*)(a & ~(uintptr_t)3);
          sh[u] = (int)(a & 3u);
          const int last = (sh[u] + nv[u] - 1) >> 2;  // last dword holding a voxel of the row-group
#pragma unroll
          for (int j = 0; j < 9; ++j)
            if (j <= last) d[u][j] = q[j];
        }
      }
#pragma unroll
      for (int u = 0; u < kLoadBatch; ++u) {
        const int idx = base + u * kBrickThreads;
        if (idx >= n) continue;
        uint32_t bits = 0u;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          bits |= in4(__builtin_amdgcn_alignbyte(d[u][j + 1], d[u][j], (uint32_t)sh[u]), label4) << (4 * j);
        s_bits[idx] = nv[u] >= 32 ? bits : bits & ((1u << nv[u]) - 1u);
      }
    }
  } else {
    // float32: a row-group is 128 B; two of them are in flight per thread
    // before either is converted
    constexpr int kLoadBatch = 2;
    for (int base = threadIdx.x; base < n; base += kBrickThreads * kLoadBatch) {
      float v[kLoadBatch][32];
      int nv[kLoadBatch];
#pragma unroll
      for (int h = 0; h < kLoadBatch; ++h) {
        const int idx = base + h * kBrickThreads;
        const char* ptr = nullptr;
        nv[h] = 0;
#pragma unroll
        for (int i = 0; i < 32; ++i) v[h][i] = 0.0f;
        if (idx < n) {
          const int p = (int)fdiv((unsigned int)idx, R.mNW, R.shNW);
          ptr = row_span<DT>(R, T, p, T.rg0 - 1 + idx - p * T.nw, nv[h]);
        }
        const float* f = (const float*)ptr;
        if (nv[h] == 32 && (((uintptr_t)ptr) & 15u) == 0) {
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const float4 q = ((const float4*)f)[i];
            v[h][4 * i] = q.x;
            v[h][4 * i + 1] = q.y;
            v[h][4 * i + 2] = q.z;
            v[h][4 * i + 3] = q.w;
          }
        } else if (nv[h] > 0) {
#pragma unroll
          for (int i = 0; i < 32; ++i)
            if (i < nv[h]) v[h][i] = f[i];
        }
      }
#pragma unroll
      for (int h = 0; h < kLoadBatch; ++h) {
        const int idx = base + h * kBrickThreads;
        if (idx >= n) continue;
        uint32_t bits = 0u;
#pragma unroll
        for (int i = 0; i < 32; ++i) bits |= (uint32_t)(v[h][i] > 0.5f) << i;
        s_bits[idx] = bits;
      }
    }
  }
}

// Thread coordinates inside a brick.
struct Lane {
  int y, l;        // cube row (voxel rows y, y+1) and 32-cube group
  uint32_t vmask;  // cubes of this group inside [-1, d2 - 1]
  bool valid;
};

// Cubes of 32-cube group l inside the ROI: cube x = 32l - 1 + k is valid iff
// k <= d2 - 32l.
__device__ inline uint32_t lane_vmask(const Roi& R, int l) {
  const int kmax = R.d[2] - 32 * l;
  return kmax >= 31 ? 0xffffffffu : ((1u << (kmax + 1)) - 1u);
}

__device__ inline Lane lane_of(const Roi& R, const Tile& T, int tid) {
  Lane L;
  const int rg = T.rg0 + tid;
  L.valid = rg < R.nrg;
  const int ry = L.valid ? (int)fdiv((unsigned int)rg, R.mG, R.shG) : 0;
  L.l = L.valid ? rg - ry * R.G : 0;
  L.y = ry - 1;
  L.vmask = lane_vmask(R, L.l);
  return L;
}

// Corner masks of the 32 cubes between voxel planes z (rows r0*) and z + 1
// (rows r1*); corner c = 4*dz + 2*dy + dx.
struct Corners {
  uint32_t c[8];
};

__device__ inline Corners make_corners(uint32_t r00, uint32_t x00, uint32_t r01, uint32_t x01, uint32_t r10,
                                       uint32_t x10, uint32_t r11, uint32_t x11) {
  Corners C;
  C.c[0] = (r00 << 1) | x00;
  C.c[1] = r00;
  C.c[2] = (r01 << 1) | x01;
  C.c[3] = r01;
  C.c[4] = (r10 << 1) | x10;
  C.c[5] = r10;
  C.c[6] = (r11 << 1) | x11;
  C.c[7] = r11;
  return C;
}

// Corner masks of plane pair (p, p+1) of the tile for thread tid.
__device__ inline Corners tile_corners(const uint32_t* s_bits, const Tile& T, const Lane& L, int p, int tid, int G) {
  uint32_t r[2][2], x[2][2];
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy) {
      const int w = (p + dz) * T.nw + tid + 1 + dy * G;
      r[dz][dy] = s_bits[w];
      x[dz][dy] = L.l > 0 ? (s_bits[w - 1] >> 31) : 0u;
    }
  return make_corners(r[0][0], x[0][0], r[0][1], x[0][1], r[1][0], x[1][0], r[1][1], x[1][1]);
}

// Count, sum of bit positions b and sum of b^2 over the set bits of w.  With
// M_k the bits whose position has bit k set, b = sum_k 2^k [b in M_k], so
// sum b = sum_k 2^k popc(w & M_k) and sum b^2 = sum_k 4^k popc(w & M_k)
// + sum_{k<l} 2^(k+l+1) popc(w & M_k & M_l).
struct WordMom {
  int c, b1, b2;
};

__device__ inline WordMom word_moments(uint32_t w) {
  WordMom m;
  if (w == 0u) {
    m.c = m.b1 = m.b2 = 0;
    return m;
  }
  if (w == 0xffffffffu) {  // 32 bits: sum b = 496, sum b^2 = 10416
    m.c = 32;
    m.b1 = 496;
    m.b2 = 10416;
    return m;
  }
  const uint32_t M[5] = {0xaaaaaaaau, 0xccccccccu, 0xf0f0f0f0u, 0xff00ff00u, 0xffff0000u};
  m.c = __popc(w);
  int b1 = 0, b2 = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const uint32_t wk = w & M[k];
    const int pk = __popc(wk);
    b1 += pk << k;
    b2 += pk << (2 * k);
#pragma unroll
    for (int l = k + 1; l < 5; ++l) b2 += __popc(wk & M[l]) << (k + l + 1);
  }
  m.b1 = b1;
  m.b2 = b2;
  return m;
}

__device__ inline int case_of(const Corners& C, int k) {
  int cas = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) cas |= (int)((C.c[c] >> k) & 1u) << c;
  return cas;
}

// ---------------------------------------------------------------------------
// Binary masks: area of each case's triangles for each ROI's spacing (one
// workgroup per ROI, one thread per case), read by every brick of the ROI.

__device__ inline double case_area_of(const Roi& R, int c) {
  const int nt = MC_NTRI[c];
  double a = 0.0;
  for (int t = 0; t < nt; ++t) {
    const double n0 = R.s[1] * R.s[2] * MC_TRI_N[c][t][0];
    const double n1 = R.s[0] * R.s[2] * MC_TRI_N[c][t][1];
    const double n2 = R.s[0] * R.s[1] * MC_TRI_N[c][t][2];
    a += 0.125 * sqrt(n0 * n0 + n1 * n1 + n2 * n2);
  }
  return a;
}

__global__ __launch_bounds__(256) void k_case_area(const Roi* __restrict__ rois, int n_rois,
                                                   double* __restrict__ case_area) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  case_area[i] = case_area_of(rois[blockIdx.x], (int)threadIdx.x);
  case_hist(case_area, n_rois)[i] = 0ull;
}

// The small-mesh path's first launch (one workgroup): the ROI record, the
// cleared staged-row count and pair-kernel accumulators, and (binary masks)
// the per-case areas and cleared case counts.
__global__ __launch_bounds__(256) void k_small_head(Roi R, Roi* __restrict__ rois, long long* __restrict__ totals,
                                                    SmallAcc* __restrict__ acc, double* __restrict__ case_area) {
  if (threadIdx.x == 0) {
    rois[0] = R;
    totals[8] = 0;
    SmallAcc A;
    for (int g = 0; g < 4; ++g) {
      A.gmax[g] = 0ull;
      A.key[g] = ~0ull;
    }
    A.pairs2d = 0ull;
    A.ticket = 0u;
    A.pad_ = 0u;
    *acc = A;
  }
  if (case_area) {
    case_area[threadIdx.x] = case_area_of(R, (int)threadIdx.x);
    case_hist(case_area, 1)[threadIdx.x] = 0ull;
  }
}

// ---------------------------------------------------------------------------
// The mesh pass: one read of the volume per brick gives its vertex and
// triangle counts, area, volume, bounding box and moments, and writes the
// canonical keys of its vertices (and soft masks' interpolation parameters)
// to a staging list, at a range of rows the brick reserves with one atomic
// (below `tmp_cap` rows; totals[8] counts them all).  Within a brick the order
// is (thread, plane, axis, cube); the row pass then places each brick's rows
// at its offset in brick order, so the final order does not depend on the
// order of the reservations.

// Binary masks: at most 80 VGPRs, so that six bricks share a CU and the
// 1,330 bricks of a 300 x 512 x 512 volume run in one round on 256 CUs (a few
// registers spill; measured faster than 96 VGPRs and five bricks per CU).
// Soft masks: at most 128 VGPRs (four bricks per CU instead of three; a few
// registers spill, measured slightly faster).
template <int DT>
__global__ __launch_bounds__(kBrickThreads, DT == 0 ? 6 : 4) void k_mesh_pass(const Roi* __restrict__ rois, int n_rois,
                                                             long long nbricks, double* __restrict__ case_area,
                                                             BrickPart* __restrict__ part,
                                                             unsigned long long* __restrict__ tmpkey,
                                                             double* __restrict__ tmpt, long long tmp_cap,
                                                             long long* __restrict__ totals, int moments,
                                                             const int* __restrict__ bmap) {
  extern __shared__ uint32_t s_bits[];
  __shared__ unsigned int s_hist[256];  // binary masks: active cubes per case
  __shared__ int s_tk[256];
  __shared__ int s_tm[256];
  __shared__ __align__(16) uint32_t s_items[kMeshItems];
  __shared__ uint32_t s_ly[kBrickThreads];  // (y + 1) | l << 20 of each thread's row-group
  __shared__ int s_scan[4];
  __shared__ uint32_t s_mx[4];
  __shared__ double s_rd[2][4];
  __shared__ long long s_rl[4];
  __shared__ int s_ri[8][4];
  __shared__ long long s_mom[10][4];
  __shared__ long long s_base;

  const long long brick = xcd_remap(blockIdx.x, nbricks);
  const int roi = bmap ? bmap[brick] : find_roi(rois, n_rois, brick);
  if (roi < 0) return;
  const Roi R = rois[roi];
  // a grid sized by a bound (ROI table planned on the device) ends past the last brick
  if (brick >= R.brick_end) return;
  const int tid = threadIdx.x;
  {
    const int c = tid;
    const int nt = MC_NTRI[c];
    s_hist[c] = 0u;
    s_tk[c] = nt | ((MC_CASE_KAPPA[c] + 128) << 8);
    s_tm[c] = (MC_CASE_M[c][0] + 128) | ((MC_CASE_M[c][1] + 128) << 8) | ((MC_CASE_M[c][2] + 128) << 16);
  }
  __syncthreads();

  const Tile T = tile_of(R, brick - R.brick_begin);
  load_tile<DT>(R, T, s_bits);
  __syncthreads();
  const Lane L = lane_of(R, T, tid);
  s_ly[tid] = (uint32_t)(L.y + 1) | ((uint32_t)L.l << 20);  // read back by the dense loop (after a barrier)
  int nv = 0, nt = 0;
  double area = 0.0, vol_d = 0.0;
  long long vol_i = 0;
  int bb[6] = {INT_MAX, INT_MAX, INT_MAX, INT_MIN, INT_MIN, INT_MIN};
  // origin of the soft tetrahedron sum: the array centre (as the FP64 oracle uses)
  const double o0 = 0.5 * R.d[0] * R.s[0], o1 = 0.5 * R.d[1] * R.s[1], o2 = 0.5 * R.d[2] * R.s[2];

  // All planes of the brick at once: each thread first classifies its 32
  // cubes of every plane pair (voxel rows held in registers, each read from
  // LDS once) into a word of active cubes and three words of crossing edges
  // per plane; the brick's active cubes, then its crossing edges, are then
  // enumerated densely over the whole workgroup (mark_words), so that a lane
  // whose cubes all touch the surface does not hold up its wave and the brick
  // takes a few barriers instead of a few per plane.
  // bit counts of the words (active cubes of plane p: byte p of actc; edges
  // along axis a of plane p, from each cube's corner 0: byte 3p + a of edc);
  // the words themselves are recomputed from the tile when they are listed
  uint32_t actc[(kTZ + 3) / 4] = {};
  uint32_t edc[(3 * kTZ + 3) / 4] = {};
  int cnt = 0, cnt_e = 0;
  long long mom[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  {
    // voxel rows y and y + 1 (and the bit before each) of the current voxel
    // plane and the next one, read from the tile one plane at a time
    uint32_t r0[2] = {0u, 0u}, x0[2] = {0u, 0u};
    auto plane_rows = [&](int p, uint32_t* r, uint32_t* x) {
#pragma unroll
      for (int dy = 0; dy < 2; ++dy) {
        r[dy] = 0u;
        x[dy] = 0u;
        if (L.valid && p < T.np) {
          const int w = p * T.nw + tid + 1 + dy * R.G;
          r[dy] = s_bits[w];
          x[dy] = L.l > 0 ? (s_bits[w - 1] >> 31) : 0u;
        }
      }
    };
    plane_rows(0, r0, x0);
#pragma unroll
    for (int p = 0; p < kTZ; ++p) {
      uint32_t r1[2], x1[2];
      plane_rows(p + 1, r1, x1);
      uint32_t act = 0u, ed[3] = {0u, 0u, 0u};
      if (L.valid && p + 1 < T.np) {
        const Corners C = make_corners(r0[0], x0[0], r0[1], x0[1], r1[0], x1[0], r1[1], x1[1]);
        uint32_t any = 0u, all = 0xffffffffu;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          any |= C.c[c];
          all &= C.c[c];
        }
        ed[0] = (C.c[0] ^ C.c[4]) & L.vmask;
        ed[1] = (C.c[0] ^ C.c[2]) & L.vmask;
        ed[2] = (C.c[0] ^ C.c[1]) & L.vmask;
        const uint32_t active = any & ~all & L.vmask;
        if (active) {
          const int z = T.pz0 - 1 + p;
          bb[0] = min(bb[0], z);
          bb[1] = min(bb[1], L.y);
          bb[2] = min(bb[2], 32 * L.l - 1 + (__ffs(active) - 1));
          bb[3] = max(bb[3], z);
          bb[4] = max(bb[4], L.y);
          bb[5] = max(bb[5], 32 * L.l - 1 + (31 - __clz(active)));
        }
        act = active;
      }
      const uint32_t ca = (uint32_t)__popc(act);
      actc[p >> 2] |= ca << (8 * (p & 3));
      cnt += (int)ca;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const uint32_t ce = (uint32_t)__popc(ed[a]);
        edc[(3 * p + a) >> 2] |= ce << (8 * ((3 * p + a) & 3));
        cnt_e += (int)ce;
      }
#pragma unroll
      for (int dy = 0; dy < 2; ++dy) {
        r0[dy] = r1[dy];
        x0[dy] = x1[dy];
      }
    }
  }
  // the brick's staged rows: one reservation
  int total_e;
  const int off_e = block_excl_scan256(cnt_e, s_scan, total_e);
  nv = cnt_e;
  if (tid == 0)
    s_base = total_e ? (long long)atomicAdd((unsigned long long*)&totals[8], (unsigned long long)total_e) : 0;
  int total;
  const int off = block_excl_scan256(cnt, s_scan, total);
  for (int c0 = 0; c0 < total; c0 += kMeshItems) {
    const int n = min(kMeshItems, total - c0);
    mark_words<kTZ>(actc, off, c0, n, s_items, s_mx);
    for (int i = tid; i < n; i += kBrickThreads) {
      const uint32_t mk = s_items[i];
      const int p = (int)(mk & 255u), t = (int)((mk >> 8) & 255u);
      const int z = T.pz0 - 1 + p;
      const uint32_t ly = s_ly[t];
      Lane Lt;
      Lt.y = (int)(ly & 0xfffffu) - 1;
      Lt.l = (int)(ly >> 20);
      const Corners C = tile_corners(s_bits, T, Lt, p, t, R.G);
      uint32_t any = 0u, all = 0xffffffffu;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        any |= C.c[c];
        all &= C.c[c];
      }
      const int k = nth_set_bit(any & ~all & lane_vmask(R, Lt.l), marker_rank(mk, i));
      const int cas = case_of(C, k);
      const int y = Lt.y, x = 32 * Lt.l - 1 + k;
      const int tk = s_tk[cas];
      nt += tk & 0xff;
      if (DT == 0) {
        const int tm = s_tm[cas];
        atomicAdd(&s_hist[cas], 1u);
        vol_i += (long long)((tk >> 8) - 128) +
                 2ll * ((long long)z * ((tm & 0xff) - 128) + (long long)y * (((tm >> 8) & 0xff) - 128) +
                        (long long)x * (((tm >> 16) & 0xff) - 128));
      } else {
        double pc[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) pc[c] = soft_value(R, z + ((c >> 2) & 1), y + ((c >> 1) & 1), x + (c & 1));
        const int ntri = tk & 0xff;
        for (int tr = 0; tr < ntri; ++tr) {
          double P[3][3];
#pragma unroll
          for (int v = 0; v < 3; ++v) {
            const int e = MC_TRI[cas][tr][v];
            const int ax = MC_EDGE_AXIS[e], k0 = MC_EDGE_C0[e];
            const int k1 = k0 | (4 >> ax);
            // the area and volume terms only (the vertex rows take the edge
            // pass's correctly rounded quotient): a reciprocal estimate refined
            // by Newton steps is within a unit in the last place
            const double tt = (0.5 - sel8d(pc, k0)) * rcp64(sel8d(pc, k1) - sel8d(pc, k0));
            const int u0 = z + ((k0 >> 2) & 1), u1 = y + ((k0 >> 1) & 1), u2 = x + (k0 & 1);
            P[v][0] = ((double)u0 + (ax == 0 ? tt : 0.0)) * R.s[0] - o0;
            P[v][1] = ((double)u1 + (ax == 1 ? tt : 0.0)) * R.s[1] - o1;
            P[v][2] = ((double)u2 + (ax == 2 ? tt : 0.0)) * R.s[2] - o2;
          }
          const double e1x = P[1][0] - P[0][0], e1y = P[1][1] - P[0][1], e1z = P[1][2] - P[0][2];
          const double e2x = P[2][0] - P[0][0], e2y = P[2][1] - P[0][1], e2z = P[2][2] - P[0][2];
          const double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
          area += 0.5 * sqrt(nx * nx + ny * ny + nz * nz);
          const double bcx = P[1][1] * P[2][2] - P[1][2] * P[2][1];
          const double bcy = P[1][2] * P[2][0] - P[1][0] * P[2][2];
          const double bcz = P[1][0] * P[2][1] - P[1][1] * P[2][0];
          vol_d += (P[0][0] * bcx + P[0][1] * bcy + P[0][2] * bcz) / 6.0;
        }
      }
    }
    __syncthreads();
  }

  __syncthreads();
  const long long base = s_base;
  for (int c0 = 0; c0 < total_e; c0 += kMeshItems) {
    const int n = min(kMeshItems, total_e - c0);
    mark_words<3 * kTZ>(edc, off_e, c0, n, s_items, s_mx);
    for (int i = tid; i < n; i += kBrickThreads) {
      const uint32_t mk = s_items[i];
      const int j = (int)(mk & 255u), t = (int)((mk >> 8) & 255u);
      const int p = j / 3, a = j - 3 * p;
      const uint32_t ly = s_ly[t];
      const int l = (int)(ly >> 20);
      // the thread's edge word (corner 0 against the corner one step along a)
      const int w0 = p * T.nw + t + 1;
      const int wq = a == 0 ? w0 + T.nw : (a == 1 ? w0 + R.G : w0);
      const uint32_t r0 = s_bits[w0], rq = s_bits[wq];
      const uint32_t x0 = l > 0 ? (s_bits[w0 - 1] >> 31) : 0u, xq = l > 0 ? (s_bits[wq - 1] >> 31) : 0u;
      const uint32_t cq = a == 2 ? r0 : ((rq << 1) | xq);
      const int k = nth_set_bit((((r0 << 1) | x0) ^ cq) & lane_vmask(R, l), marker_rank(mk, i));
      const int u0 = T.pz0 - 1 + p, u1 = (int)(ly & 0xfffffu) - 1, u2 = 32 * l - 1 + k;
      const long long row = base + c0 + i;
      if (row < tmp_cap) {
        tmpkey[row] = pack_key(u0, u1, u2, a);
        if (DT == 1) {
          const double pa = soft_value(R, u0, u1, u2);
          const double pb = soft_value(R, u0 + (a == 0), u1 + (a == 1), u2 + (a == 2));
          tmpt[row] = (0.5 - pa) / (pb - pa);
        }
      }
    }
    __syncthreads();
  }

  if (moments && L.valid) {
    // Inside-voxel moments, from the tile (still in LDS; computed here so that
    // their registers are not held through the enumeration): voxel row
    // (z, y) = (pz0 + p, L.y + 1), x = 32 l + bit, is the tile word of plane
    // p + 1, row-group tid + G (the far corner row of plane pair p); rows past
    // the array read as 0.
    long long n = 0, sz = 0, szz = 0, sb1 = 0, sb2 = 0, szb = 0;
#pragma unroll
    for (int p = 0; p < kTZ; ++p) {
      if (p + 1 < T.np) {
        const WordMom wm = word_moments(s_bits[(p + 1) * T.nw + tid + 1 + R.G]);
        const long long z = T.pz0 + p;
        n += wm.c;
        sz += z * wm.c;
        szz += z * z * wm.c;
        sb1 += wm.b1;
        sb2 += wm.b2;
        szb += z * wm.b1;
      }
    }
    const long long y = L.y + 1, x0 = 32ll * L.l;
    const long long sx = x0 * n + sb1;
    mom[0] = n;
    mom[1] = sz;
    mom[2] = y * n;
    mom[3] = sx;
    mom[4] = szz;
    mom[5] = y * y * n;
    mom[6] = x0 * x0 * n + 2 * x0 * sb1 + sb2;
    mom[7] = y * sz;
    mom[8] = x0 * sz + szb;
    mom[9] = y * sx;
  }

  // fixed-order block reduction
  const int lane = tid & 63, wid = tid >> 6;
  nv = wave_sum(nv);
  nt = wave_sum(nt);
  area = wave_sum(area);
  vol_d = wave_sum(vol_d);
  vol_i = wave_sum(vol_i);
  for (int k = 0; k < 3; ++k) {
    bb[k] = wave_min(bb[k]);
    bb[3 + k] = wave_max(bb[3 + k]);
  }
  if (moments)
    for (int k = 0; k < 10; ++k) mom[k] = wave_sum(mom[k]);
  if (lane == 0) {
    s_ri[0][wid] = nv;
    s_ri[1][wid] = nt;
    for (int k = 0; k < 6; ++k) s_ri[2 + k][wid] = bb[k];
    s_rd[0][wid] = area;
    s_rd[1][wid] = vol_d;
    s_rl[wid] = vol_i;
    for (int k = 0; k < 10; ++k) s_mom[k][wid] = mom[k];
  }
  __syncthreads();
  if (tid == 0) {
    BrickPart P;
    P.nv = s_ri[0][0] + s_ri[0][1] + s_ri[0][2] + s_ri[0][3];
    P.nt = s_ri[1][0] + s_ri[1][1] + s_ri[1][2] + s_ri[1][3];
    for (int k = 0; k < 3; ++k) {
      P.bb[k] = min(min(s_ri[2 + k][0], s_ri[2 + k][1]), min(s_ri[2 + k][2], s_ri[2 + k][3]));
      P.bb[3 + k] = max(max(s_ri[5 + k][0], s_ri[5 + k][1]), max(s_ri[5 + k][2], s_ri[5 + k][3]));
    }
    P.area = ((s_rd[0][0] + s_rd[0][1]) + s_rd[0][2]) + s_rd[0][3];
    P.vol_d = ((s_rd[1][0] + s_rd[1][1]) + s_rd[1][2]) + s_rd[1][3];
    P.vol_i = s_rl[0] + s_rl[1] + s_rl[2] + s_rl[3];
    for (int k = 0; k < 10; ++k) P.mom[k] = s_mom[k][0] + s_mom[k][1] + s_mom[k][2] + s_mom[k][3];
    P.stage = base;
    part[brick] = P;
  }
  if (DT == 0) {
    // the area follows from the case counts (summed per ROI in a fixed order
    // later), so it does not depend on how the ROI is cut into bricks
    const unsigned int h = s_hist[tid];
    if (h) atomicAdd(&case_hist(case_area, n_rois)[(size_t)roi * 256 + tid], (unsigned long long)h);
  }
}

// ---------------------------------------------------------------------------
// Per-ROI totals: exclusive scan of brick vertex counts (each brick's first
// row within its ROI), fixed-order sums.  One 1024-thread workgroup per ROI.

// 128-bit sum over a wave (two's complement halves, carry from the low half).
__device__ inline __int128 wave_sum_i128(__int128 v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const unsigned long long lo = (unsigned long long)v, hi = (unsigned long long)(v >> 64);
    const unsigned long long olo = __shfl_xor(lo, m, 64), ohi = __shfl_xor(hi, m, 64);
    const unsigned long long slo = lo + olo;
    const unsigned long long shi = hi + ohi + (slo < lo ? 1ull : 0ull);
    v = (__int128)(((unsigned __int128)shi << 64) | (unsigned __int128)slo);
  }
  return v;
}

// Covariance entry k (zz, yy, xx, zy, zx, yx) of the inside voxels' physical
// coordinates from exact integer moments S = (n, sums of z, y, x, of zz, yy,
// xx, of zy, zx, yx): cov_ij = s_i s_j (n S_ij - S_i S_j) / n^2, the
// numerator exact in 128 bits (n < 2^40 voxels and coordinates < 2^20 keep it
// below 2^120).
__device__ inline double cov_entry(const __int128* S, const double* sp, int k) {
  const int i = k < 3 ? k : (k == 5 ? 1 : 0);
  const int j = k < 3 ? k : (k == 3 ? 1 : 2);
  const __int128 n = S[0];
  if (n <= 0) return 0.0;
  const __int128 c = n * S[4 + k] - S[1 + i] * S[1 + j];
  return (double)c / ((double)n * (double)n) * (sp[i] * sp[j]);
}

__global__ __launch_bounds__(1024) void k_mesh_totals(const Roi* __restrict__ rois, int n_rois, long long nbricks,
                                                      int dtype, const double* __restrict__ case_area,
                                                      const BrickPart* __restrict__ part,
                                                      long long* __restrict__ brick_voff,
                                                      RoiMeta* __restrict__ meta, int moments) {
  __shared__ long long s_l[2][1024];
  __shared__ long long s_l2[1024];
  __shared__ double s_d[2][1024];
  __shared__ int s_b[6][1024];
  __shared__ __int128 s_m[10][16];
  __shared__ __int128 s_S[10];
  const int r = blockIdx.x, tid = threadIdx.x;
  const Roi R = rois[r];
  const long long b0 = R.brick_begin, b1 = R.brick_end;
  const long long n = b1 - b0;
  const long long chunk = (n + 1023) / 1024;
  const long long lo = b0 + min(n, chunk * tid), hi = b0 + min(n, chunk * (tid + 1));
  long long nv = 0, nt = 0, vi = 0;
  double area = 0.0, vd = 0.0;
  int bb[6] = {INT_MAX, INT_MAX, INT_MAX, INT_MIN, INT_MIN, INT_MIN};
  for (long long b = lo; b < hi; ++b) {
    const BrickPart P = part[b];
    nv += P.nv;
    nt += P.nt;
    vi += P.vol_i;
    area += P.area;
    vd += P.vol_d;
    for (int k = 0; k < 3; ++k) {
      bb[k] = min(bb[k], P.bb[k]);
      bb[3 + k] = max(bb[3 + k], P.bb[3 + k]);
    }
  }
  // exclusive scan of nv over threads (Hillis-Steele in shared memory)
  s_l[0][tid] = nv;
  __syncthreads();
  int src = 0;
  for (int d = 1; d < 1024; d <<= 1) {
    long long v = s_l[src][tid];
    if (tid >= d) v += s_l[src][tid - d];
    s_l[1 - src][tid] = v;
    __syncthreads();
    src = 1 - src;
  }
  long long off = s_l[src][tid] - nv;
  for (long long b = lo; b < hi; ++b) {
    brick_voff[b] = off;
    off += part[b].nv;
  }
  s_l2[tid] = s_l[src][1023];
  __syncthreads();
  // fixed-order tree reductions
  s_l[0][tid] = nt;
  s_l[1][tid] = vi;
  s_d[0][tid] = area;
  s_d[1][tid] = vd;
  for (int k = 0; k < 6; ++k) s_b[k][tid] = bb[k];
  __syncthreads();
  for (int w = 512; w >= 1; w >>= 1) {
    if (tid < w) {
      s_l[0][tid] += s_l[0][tid + w];
      s_l[1][tid] += s_l[1][tid + w];
      s_d[0][tid] += s_d[0][tid + w];
      s_d[1][tid] += s_d[1][tid + w];
      for (int k = 0; k < 3; ++k) {
        s_b[k][tid] = min(s_b[k][tid], s_b[k][tid + w]);
        s_b[3 + k][tid] = max(s_b[3 + k][tid], s_b[3 + k][tid + w]);
      }
    }
    __syncthreads();
  }
  // binary masks: the area from the case counts (s_d[1] is free for them)
  if (dtype == 0)
    binary_area_tree(case_area + (size_t)r * 256, case_hist(case_area, n_rois) + (size_t)r * 256, s_d[1]);
  if (tid == 0) {
    const long long V = s_l2[0];
    RoiMeta M;
    M.V = V;
    M.T = s_l[0][0];
    M.row_off = 0;
    M.V_pad = (V + kSegAlign - 1) / kSegAlign * kSegAlign;
    M.area = dtype == 0 ? s_d[1][0] : s_d[0][0];
    M.vol = dtype == 0 ? (double)s_l[1][0] * (R.s[0] * R.s[1] * R.s[2] / 48.0) : s_d[1][0];
    double R2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      M.bb[k] = s_b[k][0];
      M.bb[3 + k] = s_b[3 + k][0];
      if (V > 0) {
        M.center[k] = 0.5 * (double)(M.bb[k] + M.bb[3 + k] + 1) * R.s[k];
        const double h = 0.5 * (double)(M.bb[3 + k] - M.bb[k] + 1) * R.s[k];
        R2 += h * h;
      } else {
        M.center[k] = 0.0;
      }
    }
    M.R2 = R2;
    M.n_in = 0;
    for (int k = 0; k < 6; ++k) M.cov[k] = 0.0;
    meta[r] = M;
  }
  if (!moments) return;
  // exact moment sums, last (few registers are live): 128-bit per thread, per
  // wave, then over the 16 waves
  {
    __int128 m[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) m[k] = 0;
    for (long long b = lo; b < hi; ++b)
#pragma unroll
      for (int k = 0; k < 10; ++k) m[k] += (__int128)part[b].mom[k];
#pragma unroll
    for (int k = 0; k < 10; ++k) m[k] = wave_sum_i128(m[k]);
    if ((tid & 63) == 0)
#pragma unroll
      for (int k = 0; k < 10; ++k) s_m[k][tid >> 6] = m[k];
  }
  __syncthreads();
  // thread k < 10 sums moment k over the waves, then thread k < 6 forms
  // covariance entry k (one 128-bit product pair per thread)
  if (tid < 10) {
    __int128 v = 0;
    for (int w = 0; w < 16; ++w) v += s_m[tid][w];
    s_S[tid] = v;
  }
  __syncthreads();
  if (tid < 6) meta[r].cov[tid] = cov_entry(s_S, rois[r].s, tid);
  if (tid == 6) meta[r].n_in = (long long)s_S[0];
}

// Layout-0 row offsets of the ROIs (exclusive scan of V_pad) and the first
// column pair of each pruned ROI (at least prune_min_v vertices) in the 3D
// pruning pass (exclusive scan of ncol^2, ncol = ceil(V_pad / 1024)), one
// workgroup.  totals: [0] layout-0 rows, [1] largest V, [7] column pairs.
__global__ __launch_bounds__(1024) void k_roi_rows(int n_rois, RoiMeta* __restrict__ meta,
                                                   long long* __restrict__ totals, int prune_min_v) {
  __shared__ long long s[2][2][1024];
  const int tid = threadIdx.x;
  const int chunk = (n_rois + 1023) / 1024;
  const int lo = min(n_rois, chunk * tid), hi = min(n_rois, chunk * (tid + 1));
  auto npair = [&](const RoiMeta& M) -> long long {
    if (M.V < 2 || M.V < prune_min_v) return 0;
    const long long nc = (M.V_pad + kPruneSB * 32 - 1) / (kPruneSB * 32);
    return nc * nc;
  };
  long long sum = 0, np = 0, vmax = 0;
  for (int r = lo; r < hi; ++r) {
    const RoiMeta& M = meta[r];
    sum += M.V_pad;
    np += npair(M);
    vmax = max(vmax, M.V);
  }
  s[0][0][tid] = sum;
  s[1][0][tid] = np;
  __syncthreads();
  int src = 0;
  for (int d = 1; d < 1024; d <<= 1) {
    for (int q = 0; q < 2; ++q) {
      long long v = s[q][src][tid];
      if (tid >= d) v += s[q][src][tid - d];
      s[q][1 - src][tid] = v;
    }
    __syncthreads();
    src = 1 - src;
  }
  long long off = s[0][src][tid] - sum, poff = s[1][src][tid] - np;
  for (int r = lo; r < hi; ++r) {
    RoiMeta& M = meta[r];
    M.row_off = off;
    M.prune_off = poff;
    off += M.V_pad;
    poff += npair(M);
  }
  const long long rows0 = s[0][src][1023], np_total = s[1][src][1023];
  __syncthreads();
  s[0][0][tid] = vmax;
  __syncthreads();
  for (int w = 512; w >= 1; w >>= 1) {
    if (tid < w) s[0][0][tid] = max(s[0][0][tid], s[0][0][tid + w]);
    __syncthreads();
  }
  if (tid == 0) {
    totals[0] = rows0;
    totals[1] = s[0][0][0];
    totals[7] = np_total;
  }
}

// Refuses a call whose vertex rows exceed the rows the buffers were sized for
// (possible when a captured graph is replayed on new mask contents): raises
// the overflow flag and empties every ROI, so all later kernels do no work.
// Then writes each ROI's 3D segment (its layout-0 rows when it has pairs).
__global__ void k_check_capacity(int n_rois, long long rows0_cap, RoiMeta* __restrict__ meta,
                                 long long* __restrict__ totals, unsigned int* __restrict__ overflow,
                                 Seg* __restrict__ segs) {
  const bool over = totals[0] > rows0_cap;
  __syncthreads();
  for (int r = threadIdx.x; r < n_rois; r += blockDim.x) {
    if (over) {
      meta[r].V = 0;
      meta[r].V_pad = 0;
      meta[r].row_off = 0;
    }
    Seg S;
    S.row_begin = meta[r].row_off;
    S.n_rows = meta[r].V >= 2 ? (int)meta[r].V_pad : 0;
    S.group = r * 4;
    segs[r] = S;
  }
  __syncthreads();
  if (over && threadIdx.x == 0) {
    *overflow = 1u;
    totals[0] = 0;
    totals[1] = 0;
    totals[7] = 0;
  }
}

// ---------------------------------------------------------------------------
// Row layout: one workgroup per brick moves the brick's staged vertices to
// layout 0, at the ROI's first row plus the brick's offset within its ROI
// (rows in brick order, then the staging order within the brick), with the
// pair pass's operands: the position minus the ROI's centre, rounded to FP32,
// either as FP32 position blocks or as the split-f16 operand row; and the
// 16-row block tags.  The brick that holds a ROI's last vertex pads the ROI
// to a multiple of 32 rows with copies of that vertex.

__device__ inline void put_row(const Roi& R, const RoiMeta& M, long long row, unsigned long long k, double tv,
                               unsigned long long* __restrict__ key, double* __restrict__ tsoft,
                               float* __restrict__ pos, uint4* __restrict__ posh, int* __restrict__ orig,
                               long long src_row) {
  key[row] = k;
  if (tsoft) tsoft[row] = tv;
  const int u0 = (int)((k >> 40) & 0xFFFFF) - 1, u1 = (int)((k >> 20) & 0xFFFFF) - 1, u2 = (int)(k & 0xFFFFF) - 1;
  const int a = (int)((k >> 60) & 3);
  const double px = ((double)u0 + (a == 0 ? tv : 0.0)) * R.s[0] - M.center[0];
  const double py = ((double)u1 + (a == 1 ? tv : 0.0)) * R.s[1] - M.center[1];
  const double pz = ((double)u2 + (a == 2 ? tv : 0.0)) * R.s[2] - M.center[2];
  const float fx = (float)px, fy = (float)py, fz = (float)pz;
  const float fw = (float)((double)fx * fx + (double)fy * fy + (double)fz * fz);
  if (posh) {
    write_split_row(posh, row, fx, fy, fz, fw, h_scale_exp(M.R2));
  } else {
    float* blk = pos + (row >> 4) * 64 + (row & 15);
    blk[0] = fx;
    blk[16] = fy;
    blk[32] = fz;
    blk[48] = fw;
  }
  orig[row] = (int)src_row;
}

__global__ __launch_bounds__(256) void k_mesh_rows(const Roi* __restrict__ rois, int n_rois, long long nbricks,
                                                   const BrickPart* __restrict__ part,
                                                   const long long* __restrict__ brick_voff,
                                                   const RoiMeta* __restrict__ meta,
                                                   const unsigned long long* __restrict__ tmpkey,
                                                   const double* __restrict__ tmpt, long long tmp_cap,
                                                   unsigned long long* __restrict__ key, double* __restrict__ tsoft,
                                                   float* __restrict__ pos, uint4* __restrict__ posh,
                                                   int* __restrict__ orig, int* __restrict__ blkseg,
                                                   unsigned int* __restrict__ overflow, const int* __restrict__ bmap) {
  const long long brick = blockIdx.x;
  if (brick >= nbricks) return;
  const int r = bmap ? bmap[brick] : find_roi(rois, n_rois, brick);
  if (r < 0) return;
  const Roi& R = rois[r];
  if (brick >= R.brick_end) return;
  const RoiMeta& M = meta[r];
  const long long cnt = part[brick].nv, first = brick_voff[brick];
  // an emptied ROI (capacity exceeded), or a brick whose rows do not fit its ROI's count
  if (cnt == 0 || M.V == 0 || first + cnt > M.V) return;
  const long long src = part[brick].stage;
  if (src + cnt > tmp_cap) {  // staged beyond the list (a replay on larger meshes): refused
    if (threadIdx.x == 0) *overflow = 1u;
    return;
  }
  const long long dst = M.row_off + first;
  // four rows per thread at a time, their staged keys loaded together (a load
  // after a row's stores would wait for them)
  for (long long i0 = threadIdx.x; i0 < cnt; i0 += 4ll * blockDim.x) {
    unsigned long long kk[4];
    double tt[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long long i = min(i0 + (long long)u * blockDim.x, cnt - 1);
      kk[u] = tmpkey[src + i];
      tt[u] = tsoft ? tmpt[src + i] : 0.5;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long long i = i0 + (long long)u * blockDim.x;
      if (i >= cnt) break;
      const long long row = dst + i;
      put_row(R, M, row, kk[u], tt[u], key, tsoft, pos, posh, orig, row);
      if ((row & 15) == 0 || i == 0) blkseg[row >> 4] = r;  // a block shared with a neighbour gets the same tag
    }
  }
  if (first + cnt == M.V) {  // the ROI's last vertex: pad to V_pad rows with copies of it
    const long long last = M.row_off + M.V - 1;
    const unsigned long long k = tmpkey[src + cnt - 1];
    const double tv = tsoft ? tmpt[src + cnt - 1] : 0.5;
    for (long long row = M.row_off + M.V + threadIdx.x; row < M.row_off + M.V_pad; row += blockDim.x) {
      put_row(R, M, row, k, tv, key, tsoft, pos, posh, orig, last);
      if ((row & 15) == 0) blkseg[row >> 4] = r;
    }
  }
}

// Brick -> ROI map of a batch, so that a brick's workgroup finds its ROI with
// one load instead of a search of the ROI table.  Workgroup r < n_rois writes r
// over its ROI's bricks; the others write -1 over the bricks past the last ROI
// (the grid of a call planned on the device is sized by a bound).
constexpr int kBrickMapTailGroups = 64;

__global__ __launch_bounds__(256) void k_brick_map(const Roi* __restrict__ rois, int n_rois, long long nbricks,
                                                   int* __restrict__ bmap) {
  long long b0, b1, step = blockDim.x;
  int v;
  if ((int)blockIdx.x < n_rois) {
    v = (int)blockIdx.x;
    b0 = rois[v].brick_begin + threadIdx.x;
    b1 = min(rois[v].brick_end, nbricks);
  } else {
    v = -1;
    b0 = rois[n_rois - 1].brick_end + (long long)(blockIdx.x - n_rois) * blockDim.x + threadIdx.x;
    b1 = nbricks;
    step = (long long)kBrickMapTailGroups * blockDim.x;
  }
  for (long long b = b0; b < b1; b += step) bmap[b] = v;
}

// Clears the call's counters and the staged-row count (totals[8]).
__global__ void k_head_clear(unsigned int* __restrict__ counters, int n_counters, long long* __restrict__ totals) {
  for (int i = threadIdx.x; i < n_counters; i += blockDim.x) counters[i] = 0u;
  if (threadIdx.x == 0) totals[8] = 0;
}

// ---------------------------------------------------------------------------
// ROI tables built on the device.

// A caller's table of ROI descriptors (device memory) -> the mesh pass's ROI
// table, in one workgroup: each descriptor is validated (dims within the
// call's bounds, spacing finite and positive, strides that keep rows and
// planes apart, every voxel inside the allocation [base, base + alloc_elems)
// elements, a label only for uint8), its geometry filled as on the host, and
// brick and bucket offsets placed by exclusive scans.  A rejected descriptor
// becomes a 1x1x1 ROI with no bricks and status -1 (invalid argument).
// plan[0] receives the brick count, plan[1] the bucket count.
__global__ __launch_bounds__(1024) void k_plan_rois(const RoiDesc* __restrict__ in, int n, int dtype, long long md0,
                                                    long long md1, long long md2, const char* __restrict__ base,
                                                    long long alloc_elems, Roi* __restrict__ out,
                                                    long long* __restrict__ plan) {
  __shared__ long long s[2][2][1024];
  const int tid = threadIdx.x;
  const int chunk = (n + 1023) / 1024;
  const int lo = min(n, chunk * tid), hi = min(n, chunk * (tid + 1));
  const size_t elem = dtype == 0 ? 1 : 4;
  long long nbr = 0, nbu = 0;
  for (int r = lo; r < hi; ++r) {
    const RoiDesc D = in[r];
    bool ok = true;
    const long long dmax[3] = {md0, md1, md2};
    for (int k = 0; k < 3; ++k) {
      ok = ok && D.dims[k] >= 1 && D.dims[k] <= dmax[k];
      ok = ok && D.spacing[k] > 0.0 && isfinite(D.spacing[k]);
    }
    ok = ok && D.offset >= 0 && D.strides[0] >= 0 && D.strides[1] >= 0 && D.label >= 0 && D.label <= 255 &&
         (dtype == 0 || D.label == 0);
    long long st1 = 0, st0 = 0;
    if (ok) {
      st1 = D.strides[1] > 0 ? D.strides[1] : D.dims[2];
      st0 = D.strides[0] > 0 ? D.strides[0] : D.dims[1] * D.dims[2];
      ok = st1 >= D.dims[2] && st0 >= (D.dims[1] - 1) * st1 + D.dims[2];
      // the last voxel (products below 2^63: dims <= 2^20, strides checked against the allocation first)
      ok = ok && st0 < alloc_elems && st1 < alloc_elems &&
           D.offset + (D.dims[0] - 1) * st0 + (D.dims[1] - 1) * st1 + D.dims[2] <= alloc_elems;
    }
    Roi R;
    if (ok) {
      nbr += roi_fill(R, base + (size_t)D.offset * elem, D.dims, D.spacing, st0, st1, D.label);
    } else {
      const long long one[3] = {1, 1, 1};
      const double unit[3] = {1.0, 1.0, 1.0};
      (void)roi_fill(R, base, one, unit, 0, 0, 0);
      R.status = -1;
    }
    nbu += roi_buckets(R.d);
    out[r] = R;
  }
  s[0][0][tid] = nbr;
  s[1][0][tid] = nbu;
  __syncthreads();
  int src = 0;
  for (int d = 1; d < 1024; d <<= 1) {
    for (int q = 0; q < 2; ++q) {
      long long v = s[q][src][tid];
      if (tid >= d) v += s[q][src][tid - d];
      s[q][1 - src][tid] = v;
    }
    __syncthreads();
    src = 1 - src;
  }
  long long boff = s[0][src][tid] - nbr, uoff = s[1][src][tid] - nbu;
  for (int r = lo; r < hi; ++r) {
    Roi& R = out[r];
    const long long nb = R.status == 0 ? (long long)R.nzc * R.bpz : 0;
    R.brick_begin = boff;
    R.brick_end = boff + nb;
    roi_set_buckets(R, uoff);
    boff += nb;
    uoff += roi_buckets(R.d);
  }
  if (tid == 1023) {
    plan[0] = s[0][src][1023];
    plan[1] = s[1][src][1023];
  }
}

// One ROI descriptor passed by value (no host staging buffer).
__global__ void k_set_roi(Roi R, Roi* __restrict__ out) {
  if (threadIdx.x == 0) *out = R;
}

// ---------------------------------------------------------------------------
// Launchers.

size_t mesh_lds_bytes(int max_G) { return sizeof(uint32_t) * (size_t)(kTZ + 1) * (kBrickThreads + 1 + max_G); }

hipError_t launch_mesh_pass(int dtype, const Roi* rois, int n_rois, long long nbricks, int max_G,
                            double* case_area, BrickPart* part, unsigned int* counters, int n_counters,
                            unsigned long long* tmpkey, double* tmpt, long long tmp_cap, long long* totals,
                            int moments, int* bmap, hipStream_t st) {
  hipLaunchKernelGGL(k_head_clear, dim3(1), dim3(1024), 0, st, counters, n_counters, totals);
  if (nbricks <= 0) return hipGetLastError();
  if (n_rois < 2) bmap = nullptr;  // one ROI: the search is free
  if (bmap)
    hipLaunchKernelGGL(k_brick_map, dim3((unsigned)(n_rois + kBrickMapTailGroups)), dim3(256), 0, st, rois, n_rois,
                       nbricks, bmap);
  const size_t lds = mesh_lds_bytes(max_G);
  if (dtype == 0) {
    hipLaunchKernelGGL(k_case_area, dim3((unsigned)n_rois), dim3(256), 0, st, rois, n_rois, case_area);
    hipLaunchKernelGGL(k_mesh_pass<0>, dim3((unsigned)nbricks), dim3(kBrickThreads), lds, st, rois, n_rois, nbricks,
                       case_area, part, tmpkey, tmpt, tmp_cap, totals, moments, (const int*)bmap);
  } else {
    hipLaunchKernelGGL(k_mesh_pass<1>, dim3((unsigned)nbricks), dim3(kBrickThreads), lds, st, rois, n_rois, nbricks,
                       case_area, part, tmpkey, tmpt, tmp_cap, totals, moments, (const int*)bmap);
  }
  return hipGetLastError();
}

hipError_t launch_small_head(int dtype, const Roi& R, Roi* rois, long long* totals, SmallAcc* acc,
                             double* case_area, hipStream_t st) {
  hipLaunchKernelGGL(k_small_head, dim3(1), dim3(256), 0, st, R, rois, totals, acc,
                     dtype == 0 ? case_area : (double*)nullptr);
  return hipGetLastError();
}

hipError_t launch_mesh_core(int dtype, const Roi* rois, int n_rois, long long nbricks, int max_G,
                            double* case_area, BrickPart* part, unsigned long long* tmpkey, double* tmpt,
                            long long tmp_cap, long long* totals, int moments, hipStream_t st) {
  if (nbricks <= 0) return hipGetLastError();
  const size_t lds = mesh_lds_bytes(max_G);
  if (dtype == 0)
    hipLaunchKernelGGL(k_mesh_pass<0>, dim3((unsigned)nbricks), dim3(kBrickThreads), lds, st, rois, n_rois, nbricks,
                       case_area, part, tmpkey, tmpt, tmp_cap, totals, moments, (const int*)nullptr);
  else
    hipLaunchKernelGGL(k_mesh_pass<1>, dim3((unsigned)nbricks), dim3(kBrickThreads), lds, st, rois, n_rois, nbricks,
                       case_area, part, tmpkey, tmpt, tmp_cap, totals, moments, (const int*)nullptr);
  return hipGetLastError();
}

hipError_t launch_mesh_totals(const Roi* rois, int n_rois, long long nbricks, int dtype, const double* case_area,
                              const BrickPart* part, long long* brick_voff, RoiMeta* meta, long long* totals,
                              int moments, int prune_min_v, hipStream_t st) {
  hipLaunchKernelGGL(k_mesh_totals, dim3(n_rois), dim3(1024), 0, st, rois, n_rois, nbricks, dtype, case_area, part,
                     brick_voff,
                     meta, moments);
  hipLaunchKernelGGL(k_roi_rows, dim3(1), dim3(1024), 0, st, n_rois, meta, totals, prune_min_v);
  return hipGetLastError();
}

hipError_t launch_mesh_rows(const Roi* rois, int n_rois, long long nbricks, const BrickPart* part,
                            const long long* brick_voff, RoiMeta* meta, long long* totals, long long rows0_cap,
                            const unsigned long long* tmpkey, const double* tmpt, long long tmp_cap,
                            unsigned long long* key, double* tsoft, float* pos, uint4* posh, int* orig, int* blkseg,
                            Seg* segs, unsigned int* overflow, const int* bmap, hipStream_t st) {
  hipLaunchKernelGGL(k_check_capacity, dim3(1), dim3(1024), 0, st, n_rois, rows0_cap, meta, totals, overflow, segs);
  if (nbricks > 0)
    hipLaunchKernelGGL(k_mesh_rows, dim3((unsigned)nbricks), dim3(256), 0, st, rois, n_rois, nbricks, part,
                       brick_voff, meta, tmpkey, tmpt, tmp_cap, key, tsoft, pos, posh, orig, blkseg, overflow,
                       n_rois < 2 ? nullptr : bmap);
  return hipGetLastError();
}

hipError_t launch_plan_rois(const RoiDesc* in, int n, int dtype, const long long max_dims[3], const void* base,
                            long long alloc_elems, Roi* out, long long* plan, hipStream_t st) {
  hipLaunchKernelGGL(k_plan_rois, dim3(1), dim3(1024), 0, st, in, n, dtype, max_dims[0], max_dims[1], max_dims[2],
                     (const char*)base, alloc_elems, out, plan);
  return hipGetLastError();
}

hipError_t launch_set_roi(const Roi& R, Roi* out, hipStream_t st) {
  hipLaunchKernelGGL(k_set_roi, dim3(1), dim3(64), 0, st, R, out);
  return hipGetLastError();
}

}  // namespace s3d

