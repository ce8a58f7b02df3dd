// api.hip -- the C ABI (include/shape3d.h): argument checks, the per-device
// workspace, and the launch sequence of one call.
//
// Sequence of a call (all on the caller's stream):
//   mesh count -> per-ROI totals (vertex offsets, area, volume, centre)
//   -> read back the vertex count (sizes the vertex buffers)
//   -> emission -> plane buckets and work list -> MFMA pair maxima
//   -> exact FP64 refinement -> finalisation -> read back the results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/shape3d.h"
#include "s3d_launch.h"

using namespace s3d;

namespace {

thread_local std::string g_err;
std::mutex g_mu;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCK(call)                                                                                 \
  do {                                                                                              \
    hipError_t e_ = (call);                                                                         \
    if (e_ != hipSuccess) return fail(SHAPE3D_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct Buf {
  void* p = nullptr;
  size_t cap = 0;
};

struct Workspace {
  int device = -1;
  int cu_count = 0;
  Buf rois, part, brick_voff, meta, totals, key, tsoft, pos, orig, rowmax, blkseg, segs, bcnt, bcur, bsz, bflag, brow,
      bseg, ncol, colbase, cols, nitem, itembase, scan_tmp, counters, gres, cand, res, pairs2d, cand_nch, cand_chbase;
  void* host = nullptr;
  size_t host_cap = 0;
  hipEvent_t ev[8] = {};
  bool events = false;

  std::vector<Buf*> all() {
    return {&rois, &part,  &brick_voff, &meta,  &totals, &key,  &tsoft,   &pos,      &orig,     &rowmax,
            &blkseg, &segs, &bcnt,      &bcur,  &bsz,    &bflag, &brow,   &bseg,     &ncol,     &colbase,
            &cols,  &nitem, &itembase,  &scan_tmp, &counters, &gres, &cand, &res, &pairs2d, &cand_nch, &cand_chbase};
  }
};

std::map<int, Workspace*> g_ws;

int ensure(Buf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.cap >= bytes) return SHAPE3D_OK;
  size_t want = std::max(bytes, b.cap + b.cap / 2);
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
  want = (want + 255) & ~(size_t)255;
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(SHAPE3D_ENOMEM, "device allocation of " + std::to_string(want) + " bytes failed");
  }
  b.cap = want;
  return SHAPE3D_OK;
}

int ensure_host(Workspace& w, size_t bytes) {
  if (w.host_cap >= bytes) return SHAPE3D_OK;
  if (w.host) (void)hipHostFree(w.host);
  w.host = nullptr;
  w.host_cap = 0;
  if (hipHostMalloc(&w.host, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return fail(SHAPE3D_ENOMEM, "pinned host allocation failed");
  }
  w.host_cap = bytes;
  return SHAPE3D_OK;
}

int get_workspace(Workspace** out) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return fail(SHAPE3D_ENODEV, "no HIP device");
  }
  int dev = 0;
  HIPCK(hipGetDevice(&dev));
  auto it = g_ws.find(dev);
  if (it == g_ws.end()) {
    Workspace* w = new Workspace();
    w->device = dev;
    hipDeviceProp_t prop;
    HIPCK(hipGetDeviceProperties(&prop, dev));
    w->cu_count = prop.multiProcessorCount;
    for (int i = 0; i < 8; ++i) HIPCK(hipEventCreate(&w->ev[i]));
    w->events = true;
    it = g_ws.emplace(dev, w).first;
  }
  *out = it->second;
  return SHAPE3D_OK;
}

int check_args(const void* vol, int dtype, const int64_t dims[3], const double spacing[3]) {
  if (!vol || !dims || !spacing) return fail(SHAPE3D_EINVAL, "null argument");
  if (dtype != SHAPE3D_U8 && dtype != SHAPE3D_F32) return fail(SHAPE3D_EINVAL, "dtype must be SHAPE3D_U8 or SHAPE3D_F32");
  for (int k = 0; k < 3; ++k) {
    if (dims[k] < 1 || dims[k] > SHAPE3D_MAX_DIM) return fail(SHAPE3D_EINVAL, "dims out of range");
  }
  if (dims[2] > SHAPE3D_MAX_DIM2) return fail(SHAPE3D_EINVAL, "dims[2] out of range");
  for (int k = 0; k < 3; ++k) {
    if (!(spacing[k] > 0.0) || !std::isfinite(spacing[k])) return fail(SHAPE3D_EINVAL, "spacing must be finite and > 0");
  }
  const size_t elem = dtype == SHAPE3D_U8 ? 1 : 4;
  const size_t need = (size_t)dims[0] * (size_t)dims[1] * (size_t)dims[2] * elem;
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, vol) != hipSuccess) {
    (void)hipGetLastError();
    return fail(SHAPE3D_EINVAL, "volume pointer is not HIP device memory");
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(SHAPE3D_EINVAL, "volume pointer is not HIP device memory");
  void* base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, (void*)vol) == hipSuccess && base) {
    if ((const char*)vol + need > (const char*)base + size)
      return fail(SHAPE3D_EINVAL, "volume extends past the end of its allocation");
  } else {
    (void)hipGetLastError();
  }
  return SHAPE3D_OK;
}

// Host description of one ROI.
struct Plan {
  Roi roi;
  long long nbricks;
  long long n_buckets;
};

Plan make_plan(const void* vol, const int64_t dims[3], const double spacing[3]) {
  Plan P;
  Roi& R = P.roi;
  memset(&R, 0, sizeof(R));
  R.vol = vol;
  for (int k = 0; k < 3; ++k) {
    R.d[k] = (int)dims[k];
    R.s[k] = spacing[k];
  }
  R.G = (R.d[2] + 1 + 31) / 32;
  R.nrg = (R.d[1] + 1) * R.G;
  R.nzc = (R.d[0] + 1 + kTZ - 1) / kTZ;
  R.bpz = (R.nrg + kBrickThreads - 1) / kBrickThreads;
  R.brick_begin = 0;
  R.bucket_base[0] = 0;
  R.bucket_base[1] = 2ll * R.d[0] + 1;
  R.bucket_base[2] = R.bucket_base[1] + 2ll * R.d[1] + 1;
  P.nbricks = (long long)R.nzc * R.bpz;
  P.n_buckets = R.bucket_base[2] + 2ll * R.d[2] + 1;
  return P;
}

struct Sizes {
  long long V, rows0, rows_bound, seg_cap, col_cap, max_rows_seg;
};

// Steps up to and including the per-ROI totals; reads back V.
int run_mesh_totals(Workspace& w, const Plan& P, int dtype, hipStream_t st, RoiMeta* meta_h, long long* totals_h,
                    hipEvent_t ev_after = nullptr) {
  int rc;
  if ((rc = ensure(w.rois, sizeof(Roi)))) return rc;
  if ((rc = ensure(w.part, sizeof(BrickPart) * P.nbricks))) return rc;
  if ((rc = ensure(w.brick_voff, sizeof(long long) * P.nbricks))) return rc;
  if ((rc = ensure(w.meta, sizeof(RoiMeta)))) return rc;
  if ((rc = ensure(w.totals, sizeof(long long) * 16))) return rc;
  if ((rc = ensure_host(w, 1 << 16))) return rc;
  memcpy(w.host, &P.roi, sizeof(Roi));
  HIPCK(hipMemcpyAsync(w.rois.p, w.host, sizeof(Roi), hipMemcpyHostToDevice, st));
  HIPCK(launch_mesh_count(dtype, (const Roi*)w.rois.p, 1, P.nbricks, P.roi.G, (BrickPart*)w.part.p, st));
  HIPCK(launch_mesh_totals((const Roi*)w.rois.p, 1, P.nbricks, dtype, (const BrickPart*)w.part.p,
                           (long long*)w.brick_voff.p, (RoiMeta*)w.meta.p, (long long*)w.totals.p, st));
  if (ev_after) HIPCK(hipEventRecord(ev_after, st));
  char* h = (char*)w.host + 4096;
  HIPCK(hipMemcpyAsync(h, w.meta.p, sizeof(RoiMeta), hipMemcpyDeviceToHost, st));
  HIPCK(hipMemcpyAsync(h + 1024, w.totals.p, sizeof(long long) * 2, hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  memcpy(meta_h, h, sizeof(RoiMeta));
  memcpy(totals_h, h + 1024, sizeof(long long) * 2);
  return SHAPE3D_OK;
}

int ensure_vertex_bufs(Workspace& w, const Plan& P, int dtype, const RoiMeta& M, const long long* totals_h,
                       Sizes& S) {
  int rc;
  S.V = M.V;
  S.rows0 = totals_h[0];
  const long long rows2d_bound = 3 * S.V + (long long)(kSegAlign - 1) * P.n_buckets;
  S.rows_bound = (S.rows0 + rows2d_bound + kBlk - 1) / kBlk * kBlk;
  S.seg_cap = 1 + P.n_buckets;
  S.col_cap = S.seg_cap + S.rows_bound / (kJchunkBlocks * kBlk) + 1;
  S.max_rows_seg = std::max<long long>(M.V_pad, kSegAlign);
  const long long scan_n = std::max(std::max(P.n_buckets, (long long)kMaxCand), std::max(S.seg_cap, S.col_cap));
  if ((rc = ensure(w.key, sizeof(unsigned long long) * std::max<long long>(S.rows0, 1)))) return rc;
  if (dtype == SHAPE3D_F32 && (rc = ensure(w.tsoft, sizeof(double) * std::max<long long>(S.rows0, 1)))) return rc;
  if ((rc = ensure(w.pos, sizeof(float) * 4 * S.rows_bound))) return rc;
  if ((rc = ensure(w.orig, sizeof(int) * S.rows_bound))) return rc;
  if ((rc = ensure(w.rowmax, sizeof(float) * S.rows_bound))) return rc;
  if ((rc = ensure(w.blkseg, sizeof(int) * (S.rows_bound / kBlk + 1)))) return rc;
  if ((rc = ensure(w.segs, sizeof(Seg) * S.seg_cap))) return rc;
  if ((rc = ensure(w.bcnt, sizeof(unsigned int) * P.n_buckets))) return rc;
  if ((rc = ensure(w.bcur, sizeof(unsigned int) * P.n_buckets))) return rc;
  if ((rc = ensure(w.bsz, sizeof(long long) * P.n_buckets))) return rc;
  if ((rc = ensure(w.bflag, sizeof(long long) * P.n_buckets))) return rc;
  if ((rc = ensure(w.brow, sizeof(long long) * P.n_buckets))) return rc;
  if ((rc = ensure(w.bseg, sizeof(long long) * P.n_buckets))) return rc;
  if ((rc = ensure(w.ncol, sizeof(long long) * S.seg_cap))) return rc;
  if ((rc = ensure(w.colbase, sizeof(long long) * S.seg_cap))) return rc;
  if ((rc = ensure(w.cols, sizeof(Col) * S.col_cap))) return rc;
  if ((rc = ensure(w.nitem, sizeof(long long) * S.col_cap))) return rc;
  if ((rc = ensure(w.itembase, sizeof(long long) * S.col_cap))) return rc;
  if ((rc = ensure(w.scan_tmp, sizeof(long long) * scan_tmp_elems(scan_n)))) return rc;
  if ((rc = ensure(w.counters, sizeof(unsigned int) * 4))) return rc;
  if ((rc = ensure(w.gres, sizeof(GroupRes) * 4))) return rc;
  if ((rc = ensure(w.cand, sizeof(int) * kMaxCand))) return rc;
  if ((rc = ensure(w.res, sizeof(RoiResult)))) return rc;
  if ((rc = ensure(w.pairs2d, sizeof(long long)))) return rc;
  if ((rc = ensure(w.cand_nch, sizeof(long long) * kMaxCand))) return rc;
  if ((rc = ensure(w.cand_chbase, sizeof(long long) * kMaxCand))) return rc;
  return SHAPE3D_OK;
}

PairBufs pair_bufs(Workspace& w, const Plan& P, int dtype, const Sizes& S) {
  PairBufs B;
  B.rois = (const Roi*)w.rois.p;
  B.n_rois = 1;
  B.meta = (const RoiMeta*)w.meta.p;
  B.key = (const unsigned long long*)w.key.p;
  B.tsoft = dtype == SHAPE3D_F32 ? (const double*)w.tsoft.p : nullptr;
  B.pos = (float*)w.pos.p;
  B.orig = (int*)w.orig.p;
  B.rowmax = (float*)w.rowmax.p;
  B.blkseg = (int*)w.blkseg.p;
  B.segs = (Seg*)w.segs.p;
  B.rows0 = S.rows0;
  B.n_buckets = P.n_buckets;
  B.bcnt = (unsigned int*)w.bcnt.p;
  B.bcur = (unsigned int*)w.bcur.p;
  B.bsz = (long long*)w.bsz.p;
  B.bflag = (long long*)w.bflag.p;
  B.brow = (long long*)w.brow.p;
  B.bseg = (long long*)w.bseg.p;
  B.seg_cap = S.seg_cap;
  B.ncol = (long long*)w.ncol.p;
  B.colbase = (long long*)w.colbase.p;
  B.col_cap = S.col_cap;
  B.cols = (Col*)w.cols.p;
  B.nitem = (long long*)w.nitem.p;
  B.itembase = (long long*)w.itembase.p;
  B.totals = (long long*)w.totals.p;
  B.scan_tmp = (long long*)w.scan_tmp.p;
  B.counters = (unsigned int*)w.counters.p;
  B.gres = (GroupRes*)w.gres.p;
  B.cand = (int*)w.cand.p;
  B.max_rows_seg = S.max_rows_seg;
  B.rows_bound = S.rows_bound;
  B.res = (RoiResult*)w.res.p;
  B.pairs2d = (long long*)w.pairs2d.p;
  B.cand_nch = (long long*)w.cand_nch.p;
  B.cand_chbase = (long long*)w.cand_chbase.p;
  B.cu_count = w.cu_count;
  return B;
}

int run_emit(Workspace& w, const Plan& P, int dtype, hipStream_t st) {
  HIPCK(launch_mesh_emit(dtype, (const Roi*)w.rois.p, 1, P.nbricks, P.roi.G, (const BrickPart*)w.part.p,
                         (const long long*)w.brick_voff.p, (const RoiMeta*)w.meta.p, (unsigned long long*)w.key.p,
                         dtype == SHAPE3D_F32 ? (double*)w.tsoft.p : nullptr, (float*)w.pos.p, (int*)w.orig.p,
                         (float*)w.rowmax.p, (int*)w.blkseg.p, (Seg*)w.segs.p, st));
  return SHAPE3D_OK;
}

int shape3d_impl(const void* vol, int dtype, const int64_t dims[3], const double spacing[3], double out[6],
                 shape3d_stats* stats, int timing, hipStream_t st, RoiResult* raw = nullptr) {
  int rc = check_args(vol, dtype, dims, spacing);
  if (rc) return rc;
  if (!out) return fail(SHAPE3D_EINVAL, "null out");
  Workspace* wp = nullptr;
  if ((rc = get_workspace(&wp))) return rc;
  Workspace& w = *wp;
  const Plan P = make_plan(vol, dims, spacing);
  if (timing) HIPCK(hipEventRecord(w.ev[0], st));
  RoiMeta M;
  long long totals_h[2];
  if ((rc = run_mesh_totals(w, P, dtype, st, &M, totals_h, timing ? w.ev[1] : nullptr))) return rc;
  if (M.V == 0) {
    for (int f = 0; f < 6; ++f) out[f] = 0.0;
    if (stats) {
      memset(stats, 0, sizeof(*stats));
      for (int f = 0; f < 4; ++f) stats->pair_ids[f][0] = stats->pair_ids[f][1] = -1;
    }
    if (raw) {
      memset(raw, 0, sizeof(*raw));
      for (int f = 0; f < 4; ++f) raw->ids[f][0] = raw->ids[f][1] = -1;
    }
    g_err.clear();
    return SHAPE3D_EMPTY;
  }
  Sizes S;
  if ((rc = ensure_vertex_bufs(w, P, dtype, M, totals_h, S))) return rc;
  const PairBufs B = pair_bufs(w, P, dtype, S);
  if (timing) HIPCK(hipEventRecord(w.ev[7], st));
  if ((rc = run_emit(w, P, dtype, st))) return rc;
  if (timing) HIPCK(hipEventRecord(w.ev[2], st));
  HIPCK(launch_buckets(B, st));
  HIPCK(launch_init_groups(B, st));
  HIPCK(launch_fill_u32(B.counters, 0u, 2, st));
  if (timing) HIPCK(hipEventRecord(w.ev[3], st));
  HIPCK(launch_pair_maxima(B, st));
  if (timing) HIPCK(hipEventRecord(w.ev[4], st));
  HIPCK(launch_refine(B, st));
  if (timing) HIPCK(hipEventRecord(w.ev[5], st));
  HIPCK(launch_finalize(B, st));
  RoiResult* rh = (RoiResult*)((char*)w.host + 8192);
  HIPCK(hipMemcpyAsync(rh, w.res.p, sizeof(RoiResult), hipMemcpyDeviceToHost, st));
  if (timing) HIPCK(hipEventRecord(w.ev[6], st));
  HIPCK(hipStreamSynchronize(st));
  if (rh->status < 0) return fail(rh->status, "candidate rows of the exact refinement exceeded their capacity");
  for (int f = 0; f < 6; ++f) out[f] = rh->out[f];
  if (raw) *raw = *rh;
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->n_vertices = rh->V;
    stats->n_triangles = rh->T;
    for (int f = 0; f < 4; ++f) {
      stats->pair_ids[f][0] = rh->ids[f][0];
      stats->pair_ids[f][1] = rh->ids[f][1];
      stats->candidates[f] = rh->cand[f];
    }
    stats->pairs_3d = rh->V * (rh->V - 1) / 2;
    stats->pairs_2d = rh->pairs2d;
    if (timing) {
      // phases: 0 mesh count + totals, 1 emit, 2 buckets + work list, 3 MFMA pair maxima, 4 refine,
      // 5 finalise + read-back, 6 whole call (including the vertex-count read-back)
      const int a[7] = {0, 7, 2, 3, 4, 5, 0};
      const int b[7] = {1, 2, 3, 4, 5, 6, 6};
      for (int k = 0; k < 7; ++k) {
        float ms = 0.f;
        HIPCK(hipEventElapsedTime(&ms, w.ev[a[k]], w.ev[b[k]]));
        stats->ms[k] = ms;
      }
    }
  }
  g_err.clear();
  return SHAPE3D_OK;
}

}  // namespace

extern "C" {

int shape3d(const uint8_t* mask, const int64_t dims[3], const double spacing[3], double out[6]) {
  std::lock_guard<std::mutex> lk(g_mu);
  return shape3d_impl(mask, SHAPE3D_U8, dims, spacing, out, nullptr, 0, nullptr);
}

int shape3d_ex(const void* vol, int dtype, const int64_t dims[3], const double spacing[3], double out[6],
               shape3d_stats* stats, int timing, void* stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  return shape3d_impl(vol, dtype, dims, spacing, out, stats, timing, (hipStream_t)stream);
}

int shape3d_vertices(const void* vol, int dtype, const int64_t dims[3], const double spacing[3], int64_t* ids,
                     double* pos, int64_t cap, int64_t* n_out, void* stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  int rc = check_args(vol, dtype, dims, spacing);
  if (rc) return rc;
  if (!n_out || (!ids && cap > 0)) return fail(SHAPE3D_EINVAL, "null output");
  hipStream_t st = (hipStream_t)stream;
  Workspace* wp = nullptr;
  if ((rc = get_workspace(&wp))) return rc;
  Workspace& w = *wp;
  const Plan P = make_plan(vol, dims, spacing);
  RoiMeta M;
  long long totals_h[2];
  if ((rc = run_mesh_totals(w, P, dtype, st, &M, totals_h))) return rc;
  *n_out = M.V;
  if (M.V > cap) return fail(SHAPE3D_ECAPACITY, "vertex buffer too small");
  if (M.V == 0) return SHAPE3D_EMPTY;
  Sizes S;
  if ((rc = ensure_vertex_bufs(w, P, dtype, M, totals_h, S))) return rc;
  if ((rc = run_emit(w, P, dtype, st))) return rc;
  HIPCK(launch_export_vertices((const unsigned long long*)w.key.p,
                               dtype == SHAPE3D_F32 ? (const double*)w.tsoft.p : nullptr, (const RoiMeta*)w.meta.p,
                               (const Roi*)w.rois.p, (long long*)ids, pos, M.V, st));
  HIPCK(hipStreamSynchronize(st));
  g_err.clear();
  return SHAPE3D_OK;
}

int shape3d_soft_forward(const float* p, const int64_t dims[3], const double spacing[3], double out[6],
                         shape3d_soft_saved* saved, void* stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!saved) return fail(SHAPE3D_EINVAL, "null saved context");
  RoiResult raw;
  const int rc = shape3d_impl(p, SHAPE3D_F32, dims, spacing, out, nullptr, 0, (hipStream_t)stream, &raw);
  if (rc < 0) return rc;
  for (int k = 0; k < 3; ++k) {
    saved->dims[k] = dims[k];
    saved->spacing[k] = spacing[k];
  }
  for (int f = 0; f < 6; ++f) saved->features[f] = out[f];
  saved->signed_volume = raw.vol_signed;
  for (int f = 0; f < 4; ++f) {
    saved->pair_ids[f][0] = raw.ids[f][0];
    saved->pair_ids[f][1] = raw.ids[f][1];
  }
  saved->status = rc;
  return rc;
}

int shape3d_soft_backward(const float* p, const shape3d_soft_saved* saved, const double grad_out[6], float* grad_p,
                          void* stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!saved || !grad_out || !grad_p) return fail(SHAPE3D_EINVAL, "null argument");
  int rc = check_args(p, SHAPE3D_F32, saved->dims, saved->spacing);
  if (rc) return rc;
  rc = check_args(grad_p, SHAPE3D_F32, saved->dims, saved->spacing);
  if (rc) return rc;
  for (int f = 0; f < 6; ++f)
    if (!std::isfinite(grad_out[f])) return fail(SHAPE3D_EINVAL, "grad_out must be finite");
  Workspace* wp = nullptr;
  if ((rc = get_workspace(&wp))) return rc;
  SoftBwdArgs A;
  memset(&A, 0, sizeof(A));
  for (int k = 0; k < 3; ++k) {
    A.d[k] = (int)saved->dims[k];
    A.s[k] = saved->spacing[k];
    A.o[k] = 0.5 * (double)saved->dims[k] * saved->spacing[k];
  }
  for (int f = 0; f < 6; ++f) A.gout[f] = grad_out[f];
  // an empty mask has no surface: every gradient is zero
  const bool empty = saved->status == SHAPE3D_EMPTY;
  A.g_vol_signed = grad_out[0] * (saved->signed_volume >= 0.0 ? 1.0 : -1.0);
  for (int f = 0; f < 4; ++f) {
    A.D[f] = empty ? 0.0 : saved->features[2 + f];
    A.pair_ids[f][0] = saved->pair_ids[f][0];
    A.pair_ids[f][1] = saved->pair_ids[f][1];
  }
  HIPCK(launch_soft_backward(p, A, grad_p, wp->cu_count, (hipStream_t)stream));
  HIPCK(hipStreamSynchronize((hipStream_t)stream));
  g_err.clear();
  return SHAPE3D_OK;
}

const char* shape3d_last_error(void) { return g_err.c_str(); }

int shape3d_release(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_ws) {
    Workspace* w = kv.second;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(w->device);
    (void)hipDeviceSynchronize();
    for (Buf* b : w->all())
      if (b->p) (void)hipFree(b->p);
    if (w->host) (void)hipHostFree(w->host);
    for (int i = 0; i < 8; ++i)
      if (w->events) (void)hipEventDestroy(w->ev[i]);
    (void)hipSetDevice(cur);
    delete w;
  }
  g_ws.clear();
  return SHAPE3D_OK;
}

int shape3d_version(void) { return 100; }

}  // extern "C"
