// api.hip -- the C ABI (include/shape3d.h): argument checks, the per-device
// workspace, and the launch sequence of a call.
//
// Every call processes a batch of ROIs (a single ROI is a batch of one), all
// on the caller's stream:
//   mesh count -> per-ROI totals (vertex offsets, area, volume, centre)
//   -> read back the total vertex rows (sizes the vertex buffers)
//   -> capacity check -> emission -> plane buckets and work list
//   -> MFMA pair maxima -> exact FP64 refinement -> finalisation
//   -> read back the per-ROI results.
// The batched entry point can record everything after the ROI table upload as
// a hipGraph and replay it for later calls with the same layout; the capacity
// check turns a replay on larger meshes into SHAPE3D_ECAPACITY for the graph
// run, after which the call is re-run eagerly with larger buffers.
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

struct GraphRec {
  hipGraphExec_t exec = nullptr;
  long long generation = -1;
  RoiResult* host_res = nullptr;  // pinned, written by the graph's last copy
  long long n_rois = 0;
  long long stamp = 0;            // last use (the least recently used graph is dropped first)
};

constexpr size_t kMaxGraphs = 64;  // recorded batch layouts kept per device

struct Workspace {
  int device = -1;
  int cu_count = 0;
  long long generation = 0;  // bumped whenever a buffer is reallocated (graphs hold pointers)
  Buf rois, part, brick_voff, meta, totals, key, tsoft, pos, orig, rowmax, blkseg, segs, bcnt, bcur, bsz, bflag, brow,
      bseg, bgroup, ncol, colbase, cols, nitem, itembase, scan_tmp, counters, gres, cand, res, pairs2d, cand_nch, cand_chbase,
      posh, case_area, soft_rois, soft_edges, soft_field, soft_ctr, soft_blk;
  void* host = nullptr;  // pinned staging: ROI table, read-backs, results
  size_t host_cap = 0;
  hipEvent_t ev[8] = {};
  bool events = false;
  hipStream_t graph_stream = nullptr;  // graphs are recorded and replayed here (the caller's
                                       // stream may be the legacy null stream, which cannot record)
  long long rows0_cap = 0;  // layout-0 rows the vertex buffers were sized for
  long long last_rows0 = 0;  // layout-0 rows of the last eager run (a recorded graph is sized for them)
  std::map<std::string, GraphRec> graphs;
  long long stamp = 0;

  std::vector<Buf*> all() {
    return {&rois,     &part,    &brick_voff, &meta,    &totals, &key,   &tsoft, &pos,     &orig,     &rowmax,
            &blkseg,   &segs,    &bcnt,       &bcur,    &bsz,    &bflag, &brow,  &bseg,    &bgroup, &ncol,     &colbase,
            &cols,     &nitem,   &itembase,   &scan_tmp, &counters, &gres, &cand, &res,    &pairs2d,  &cand_nch,
            &cand_chbase, &posh, &case_area, &soft_rois, &soft_edges, &soft_field, &soft_ctr, &soft_blk};
  }
};

std::map<int, Workspace*> g_ws;

// Tile sizes of the pair pass for every device (results do not depend on them).
Tuning g_tune = {8, 1024, 0, 1};

bool valid_tuning(const Tuning& t) {
  return (t.itile == 2 || t.itile == 4 || t.itile == 8) &&
         (t.jchunk == 64 || t.jchunk == 128 || t.jchunk == 256 || t.jchunk == 512 || t.jchunk == 1024) && t.blocks_per_cu >= 0 &&
         t.blocks_per_cu <= 64 && (t.kernel == 0 || (t.kernel == 1 && t.itile >= 4));
}

void drop_graphs(Workspace& w) {
  for (auto& kv : w.graphs) {
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (kv.second.host_res) (void)hipHostFree(kv.second.host_res);
  }
  w.graphs.clear();
}

int ensure(Workspace& w, Buf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.cap >= bytes) return SHAPE3D_OK;
  size_t want = std::max(bytes, b.cap + b.cap / 2);
  want = (want + 255) & ~(size_t)255;
  // recorded graphs hold the old pointer: finish outstanding work and drop them
  (void)hipDeviceSynchronize();
  drop_graphs(w);
  w.generation++;
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
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
  (void)hipDeviceSynchronize();
  drop_graphs(w);
  w.generation++;
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
    HIPCK(hipStreamCreateWithFlags(&w->graph_stream, hipStreamNonBlocking));
    it = g_ws.emplace(dev, w).first;
  }
  *out = it->second;
  return SHAPE3D_OK;
}

int check_dims_spacing(const int64_t dims[3], const double spacing[3]) {
  for (int k = 0; k < 3; ++k) {
    if (dims[k] < 1 || dims[k] > SHAPE3D_MAX_DIM) return fail(SHAPE3D_EINVAL, "dims out of range");
    if (!(spacing[k] > 0.0) || !std::isfinite(spacing[k])) return fail(SHAPE3D_EINVAL, "spacing must be finite and > 0");
  }
  if (dims[2] > SHAPE3D_MAX_DIM2) return fail(SHAPE3D_EINVAL, "dims[2] out of range");
  return SHAPE3D_OK;
}

// The device allocation holding ptr: [*base, *base + *size) (*base = null if
// the runtime cannot tell).  Fails for host memory.
int device_range(const void* ptr, const char** base, size_t* size) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, ptr) != hipSuccess) {
    (void)hipGetLastError();
    return fail(SHAPE3D_EINVAL, "volume pointer is not HIP device memory");
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(SHAPE3D_EINVAL, "volume pointer is not HIP device memory");
  void* b = nullptr;
  size_t s = 0;
  if (hipMemGetAddressRange(&b, &s, (void*)ptr) == hipSuccess && b) {
    *base = (const char*)b;
    *size = s;
  } else {
    (void)hipGetLastError();
    *base = nullptr;
    *size = 0;
  }
  return SHAPE3D_OK;
}

int check_args(const void* vol, int dtype, const int64_t dims[3], const double spacing[3]) {
  if (!vol || !dims || !spacing) return fail(SHAPE3D_EINVAL, "null argument");
  if (dtype != SHAPE3D_U8 && dtype != SHAPE3D_F32) return fail(SHAPE3D_EINVAL, "dtype must be SHAPE3D_U8 or SHAPE3D_F32");
  int rc = check_dims_spacing(dims, spacing);
  if (rc) return rc;
  const size_t need = (size_t)dims[0] * (size_t)dims[1] * (size_t)dims[2] * (dtype == SHAPE3D_U8 ? 1 : 4);
  const char* base;
  size_t size;
  if ((rc = device_range(vol, &base, &size))) return rc;
  if (base && (const char*)vol + need > base + size)
    return fail(SHAPE3D_EINVAL, "volume extends past the end of its allocation");
  return SHAPE3D_OK;
}

// Host description of a batch.
struct Batch {
  std::vector<Roi> rois;
  long long nbricks = 0;
  long long n_buckets = 0;
  int max_G = 1;
  int n() const { return (int)rois.size(); }
};

// Magic numbers (fdiv) of the kernels' 32-bit division by D (numerators < 2^31).
void magic_div(unsigned int D, unsigned int& m, int& sh) {
  int k = 0;
  while ((1ull << k) < D) ++k;  // ceil(log2 D)
  sh = 31 + k;
  m = (unsigned int)((1ull << sh) / D + 1);
}

void batch_add(Batch& B, const void* vol, const int64_t dims[3], const double spacing[3]) {
  Roi R;
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
  magic_div((unsigned int)R.G, R.mG, R.shG);
  magic_div((unsigned int)(kBrickThreads + 1 + R.G), R.mNW, R.shNW);
  R.brick_begin = B.nbricks;
  R.bucket_base[0] = B.n_buckets;
  R.bucket_base[1] = R.bucket_base[0] + 2ll * R.d[0] + 1;
  R.bucket_base[2] = R.bucket_base[1] + 2ll * R.d[1] + 1;
  B.nbricks += (long long)R.nzc * R.bpz;
  B.n_buckets = R.bucket_base[2] + 2ll * R.d[2] + 1;
  B.max_G = std::max(B.max_G, R.G);
  B.rois.push_back(R);
}

struct Sizes {
  long long rows0, rows_bound, seg_cap, col_cap;
};

Sizes sizes_for(const Batch& B, long long rows0) {
  Sizes S;
  S.rows0 = rows0;
  // plane layouts: every vertex lies in one bucket per axis, each bucket padded by < 32 rows
  const long long rows2d_bound = 3 * S.rows0 + (long long)(kSegAlign - 1) * B.n_buckets;
  S.rows_bound = (S.rows0 + rows2d_bound + kBlk - 1) / kBlk * kBlk;
  S.seg_cap = B.n() + B.n_buckets;
  S.col_cap = S.seg_cap + S.rows_bound / (kMinJchunk * kBlk) + 1;
  return S;
}

// Buffers that depend only on the batch layout.
int ensure_layout_bufs(Workspace& w, const Batch& B) {
  int rc;
  const int n = B.n();
  if ((rc = ensure(w, w.rois, sizeof(Roi) * n))) return rc;
  if ((rc = ensure(w, w.part, sizeof(BrickPart) * B.nbricks))) return rc;
  if ((rc = ensure(w, w.brick_voff, sizeof(long long) * B.nbricks))) return rc;
  if ((rc = ensure(w, w.meta, sizeof(RoiMeta) * n))) return rc;
  if ((rc = ensure(w, w.case_area, sizeof(double) * 256 * (size_t)n))) return rc;
  if ((rc = ensure(w, w.totals, sizeof(long long) * 16))) return rc;
  if ((rc = ensure(w, w.counters, sizeof(unsigned int) * kCounterWords))) return rc;
  if ((rc = ensure(w, w.gres, sizeof(GroupRes) * 4 * (size_t)n))) return rc;
  if ((rc = ensure(w, w.res, sizeof(RoiResult) * n))) return rc;
  if ((rc = ensure(w, w.pairs2d, sizeof(long long) * n))) return rc;
  if ((rc = ensure(w, w.bcnt, sizeof(unsigned int) * B.n_buckets))) return rc;
  if ((rc = ensure(w, w.bcur, sizeof(unsigned int) * B.n_buckets))) return rc;
  if ((rc = ensure(w, w.bsz, sizeof(long long) * B.n_buckets))) return rc;
  if ((rc = ensure(w, w.bflag, sizeof(long long) * B.n_buckets))) return rc;
  if ((rc = ensure(w, w.brow, sizeof(long long) * B.n_buckets))) return rc;
  if ((rc = ensure(w, w.bseg, sizeof(long long) * B.n_buckets))) return rc;
  if ((rc = ensure(w, w.bgroup, sizeof(int) * B.n_buckets))) return rc;
  // pinned staging: [0, 4096) read-backs, then the ROI table, then the results
  const size_t host_need = 4096 + sizeof(Roi) * (size_t)n + 256 + sizeof(RoiResult) * (size_t)n;
  if ((rc = ensure_host(w, host_need))) return rc;
  return SHAPE3D_OK;
}

RoiResult* host_results(Workspace& w, const Batch& B) {
  const uintptr_t p = (uintptr_t)w.host + 4096 + sizeof(Roi) * (size_t)B.n();
  return (RoiResult*)((p + 255) & ~(uintptr_t)255);
}

// Buffers sized by the layout-0 row count (all ROIs' padded vertex rows).
// Grows the vertex buffers to hold rows0 layout-0 rows (they never shrink) and
// returns in S the sizes of this call's work, which follow rows0 itself.
int ensure_vertex_bufs(Workspace& w, const Batch& B, int dtype, long long rows0, Sizes& S_call) {
  int rc;
  const Sizes S = sizes_for(B, std::max<long long>(rows0, w.rows0_cap));
  S_call = sizes_for(B, rows0);
  const long long scan_n = std::max(std::max(B.n_buckets, S.rows_bound), std::max(S.seg_cap, S.col_cap));
  if ((rc = ensure(w, w.key, sizeof(unsigned long long) * std::max<long long>(S.rows0, 1)))) return rc;
  if (dtype == SHAPE3D_F32 && (rc = ensure(w, w.tsoft, sizeof(double) * std::max<long long>(S.rows0, 1)))) return rc;
  // pair-pass operands: FP32 position blocks (kernel 0, 16 B per row) or
  // split-f16 B operands (kernel 1, 1 KB per 32-row block)
  if (g_tune.kernel == 0 && (rc = ensure(w, w.pos, sizeof(float) * 4 * S.rows_bound))) return rc;
  if (g_tune.kernel == 1 && (rc = ensure(w, w.posh, (size_t)1024 * ((S.rows_bound + 31) / 32)))) return rc;
  if ((rc = ensure(w, w.orig, sizeof(int) * S.rows_bound))) return rc;
  if ((rc = ensure(w, w.rowmax, sizeof(float) * S.rows_bound))) return rc;
  if ((rc = ensure(w, w.blkseg, sizeof(int) * (S.rows_bound / kBlk + 1)))) return rc;
  if ((rc = ensure(w, w.segs, sizeof(Seg) * S.seg_cap))) return rc;
  if ((rc = ensure(w, w.ncol, sizeof(long long) * S.seg_cap))) return rc;
  if ((rc = ensure(w, w.colbase, sizeof(long long) * S.seg_cap))) return rc;
  if ((rc = ensure(w, w.cols, sizeof(Col) * S.col_cap))) return rc;
  if ((rc = ensure(w, w.nitem, sizeof(long long) * S.col_cap))) return rc;
  if ((rc = ensure(w, w.itembase, sizeof(long long) * S.col_cap))) return rc;
  if ((rc = ensure(w, w.scan_tmp, sizeof(long long) * scan_tmp_elems(scan_n)))) return rc;
  // candidate rows of the exact refinement: every row could be one
  if ((rc = ensure(w, w.cand, sizeof(int) * S.rows_bound))) return rc;
  if ((rc = ensure(w, w.cand_nch, sizeof(long long) * S.rows_bound))) return rc;
  if ((rc = ensure(w, w.cand_chbase, sizeof(long long) * S.rows_bound))) return rc;
  w.rows0_cap = S.rows0;
  return SHAPE3D_OK;
}

PairBufs pair_bufs(Workspace& w, const Batch& Bt, int dtype, const Sizes& S) {
  PairBufs B;
  B.rois = (const Roi*)w.rois.p;
  B.n_rois = Bt.n();
  B.meta = (const RoiMeta*)w.meta.p;
  B.key = (const unsigned long long*)w.key.p;
  B.tsoft = dtype == SHAPE3D_F32 ? (const double*)w.tsoft.p : nullptr;
  B.pos = (float*)w.pos.p;
  B.posh = (uint4*)w.posh.p;
  B.orig = (int*)w.orig.p;
  B.rowmax = (float*)w.rowmax.p;
  B.blkseg = (int*)w.blkseg.p;
  B.segs = (Seg*)w.segs.p;
  B.rows0 = S.rows0;
  B.n_buckets = Bt.n_buckets;
  B.bcnt = (unsigned int*)w.bcnt.p;
  B.bcur = (unsigned int*)w.bcur.p;
  B.bsz = (long long*)w.bsz.p;
  B.bflag = (long long*)w.bflag.p;
  B.bgroup = (int*)w.bgroup.p;
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
  B.cand_cap = S.rows_bound;
  B.tune = g_tune;
  B.max_rows_seg = S.rows0;
  B.rows_bound = S.rows_bound;
  B.res = (RoiResult*)w.res.p;
  B.pairs2d = (long long*)w.pairs2d.p;
  B.cand_nch = (long long*)w.cand_nch.p;
  B.cand_chbase = (long long*)w.cand_chbase.p;
  B.cu_count = w.cu_count;
  return B;
}

// Mesh count and per-ROI totals (launches only).
int launch_head(Workspace& w, const Batch& Bt, int dtype, hipStream_t st) {
  HIPCK(launch_fill_u32((unsigned int*)w.counters.p, 0u, kCounterWords, st));
  HIPCK(launch_mesh_count(dtype, (const Roi*)w.rois.p, Bt.n(), Bt.nbricks, Bt.max_G, (double*)w.case_area.p,
                          (BrickPart*)w.part.p, st));
  HIPCK(launch_mesh_totals((const Roi*)w.rois.p, Bt.n(), Bt.nbricks, dtype, (const BrickPart*)w.part.p,
                           (long long*)w.brick_voff.p, (RoiMeta*)w.meta.p, (long long*)w.totals.p, st));
  return SHAPE3D_OK;
}

// Everything after the totals (launches only).  ev: optional phase events
// recorded before emission, buckets, pairs, refinement and finalisation.
int launch_tail(Workspace& w, const Batch& Bt, int dtype, const Sizes& S, hipStream_t st, RoiResult* host_res,
                hipEvent_t* ev) {
  const PairBufs B = pair_bufs(w, Bt, dtype, S);
  HIPCK(launch_check_capacity(Bt.n(), S.rows0, (RoiMeta*)w.meta.p, (long long*)w.totals.p,
                              (unsigned int*)w.counters.p + 2, st));
  if (ev) HIPCK(hipEventRecord(ev[0], st));
  HIPCK(launch_mesh_emit(dtype, (const Roi*)w.rois.p, Bt.n(), Bt.nbricks, Bt.max_G, (const BrickPart*)w.part.p,
                         (const long long*)w.brick_voff.p, (const RoiMeta*)w.meta.p,
                         (const unsigned int*)w.counters.p + 2, (unsigned long long*)w.key.p,
                         dtype == SHAPE3D_F32 ? (double*)w.tsoft.p : nullptr, (float*)w.pos.p, split_rows(B),
                         (int*)w.orig.p, (int*)w.blkseg.p, (Seg*)w.segs.p, st));
  if (ev) HIPCK(hipEventRecord(ev[1], st));
  HIPCK(launch_buckets(B, st));
  HIPCK(launch_init_groups(B, st));  // also zeroes the row maxima
  if (ev) HIPCK(hipEventRecord(ev[2], st));
  HIPCK(launch_pair_maxima(B, st));
  if (ev) HIPCK(hipEventRecord(ev[3], st));
  HIPCK(launch_refine(B, st));
  if (ev) HIPCK(hipEventRecord(ev[4], st));
  HIPCK(launch_finalize(B, st));
  HIPCK(hipMemcpyAsync(host_res, w.res.p, sizeof(RoiResult) * Bt.n(), hipMemcpyDeviceToHost, st));
  return SHAPE3D_OK;
}

// One eager run of a batch; results land in host_res (pinned, one per ROI).
int run_eager(Workspace& w, const Batch& Bt, int dtype, hipStream_t st, RoiResult* host_res, int timing,
              float* phase_ms) {
  int rc;
  char* h = (char*)w.host;
  memcpy(h + 4096, Bt.rois.data(), sizeof(Roi) * Bt.n());
  HIPCK(hipMemcpyAsync(w.rois.p, h + 4096, sizeof(Roi) * Bt.n(), hipMemcpyHostToDevice, st));
  if (timing) HIPCK(hipEventRecord(w.ev[0], st));
  if ((rc = launch_head(w, Bt, dtype, st))) return rc;
  if (timing) HIPCK(hipEventRecord(w.ev[1], st));
  long long* th = (long long*)h;
  HIPCK(hipMemcpyAsync(th, w.totals.p, sizeof(long long) * 2, hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  Sizes S;
  if ((rc = ensure_vertex_bufs(w, Bt, dtype, th[0], S))) return rc;
  w.last_rows0 = th[0];
  if ((rc = launch_tail(w, Bt, dtype, S, st, host_res, timing ? &w.ev[2] : nullptr))) return rc;
  if (timing) HIPCK(hipEventRecord(w.ev[7], st));
  HIPCK(hipStreamSynchronize(st));
  if (timing && phase_ms) {
    // 0 mesh count + totals, 1 emit, 2 buckets + work list, 3 MFMA pair maxima, 4 refine,
    // 5 finalise + read-back, 6 whole call (including the row-count read-back)
    const int a[7] = {0, 2, 3, 4, 5, 6, 0};
    const int b[7] = {1, 3, 4, 5, 6, 7, 7};
    for (int k = 0; k < 7; ++k) HIPCK(hipEventElapsedTime(&phase_ms[k], w.ev[a[k]], w.ev[b[k]]));
  }
  return SHAPE3D_OK;
}

void fill_stats(shape3d_stats* stats, const RoiResult& R, const float* ms) {
  if (!stats) return;
  memset(stats, 0, sizeof(*stats));
  stats->n_vertices = R.V;
  stats->n_triangles = R.T;
  for (int f = 0; f < 4; ++f) {
    stats->pair_ids[f][0] = R.ids[f][0];
    stats->pair_ids[f][1] = R.ids[f][1];
    stats->candidates[f] = R.cand[f];
  }
  stats->pairs_3d = R.V * (R.V - 1) / 2;
  stats->pairs_2d = R.pairs2d;
  if (ms)
    for (int k = 0; k < 7; ++k) stats->ms[k] = ms[k];
}

int shape3d_impl(const void* vol, int dtype, const int64_t dims[3], const double spacing[3], double out[6],
                 shape3d_stats* stats, int timing, hipStream_t st, RoiResult* raw = nullptr) {
  int rc = check_args(vol, dtype, dims, spacing);
  if (rc) return rc;
  if (!out) return fail(SHAPE3D_EINVAL, "null out");
  Workspace* wp = nullptr;
  if ((rc = get_workspace(&wp))) return rc;
  Workspace& w = *wp;
  Batch Bt;
  batch_add(Bt, vol, dims, spacing);
  if ((rc = ensure_layout_bufs(w, Bt))) return rc;
  RoiResult* hres = host_results(w, Bt);
  float ms[8] = {0};
  if ((rc = run_eager(w, Bt, dtype, st, hres, timing, ms))) return rc;
  if (hres->status < 0) return fail(hres->status, "an internal capacity was exceeded");
  for (int f = 0; f < 6; ++f) out[f] = hres->out[f];
  if (raw) *raw = *hres;
  fill_stats(stats, *hres, timing ? ms : nullptr);
  g_err.clear();
  return hres->status;
}

std::string layout_signature(const void* base, int dtype, const shape3d_roi* rois, int64_t n) {
  std::string sig((const char*)&base, sizeof(base));
  sig.append((const char*)&dtype, sizeof(dtype));
  sig.append((const char*)rois, sizeof(shape3d_roi) * (size_t)n);
  return sig;
}

// Records launch_head + launch_tail for the batch as a graph (buffers already sized).
int capture_graph(Workspace& w, const Batch& Bt, int dtype, hipStream_t st, GraphRec& rec) {
  rec.n_rois = Bt.n();
  if (hipHostMalloc((void**)&rec.host_res, sizeof(RoiResult) * Bt.n(), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    rec.host_res = nullptr;
    return fail(SHAPE3D_ENOMEM, "pinned host allocation failed");
  }
  // sized for the eager run just made: a replay that finds more rows than
  // that is caught by the capacity check and re-run eagerly
  const Sizes S = sizes_for(Bt, w.last_rows0);
  hipGraph_t graph = nullptr;
  HIPCK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  int rc = launch_head(w, Bt, dtype, st);
  if (!rc) rc = launch_tail(w, Bt, dtype, S, st, rec.host_res, nullptr);
  const hipError_t ec = hipStreamEndCapture(st, &graph);
  if (rc || ec != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc ? rc : fail(SHAPE3D_EHIP, std::string("graph capture failed: ") + hipGetErrorString(ec));
  }
  const hipError_t ei = hipGraphInstantiate(&rec.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) {
    rec.exec = nullptr;
    return fail(SHAPE3D_EHIP, std::string("graph instantiation failed: ") + hipGetErrorString(ei));
  }
  rec.generation = w.generation;
  return SHAPE3D_OK;
}

// The batched forward pass; on success *hres_out points at the per-ROI results
// (pinned host memory owned by the workspace, valid until the next call).
// Validates a ROI table against the allocation holding base and builds the batch.
int make_batch(const void* base, int dtype, const shape3d_roi* rois, int64_t n_rois, Batch& Bt) {
  if (!base || !rois || n_rois < 1) return fail(SHAPE3D_EINVAL, "null argument or empty batch");
  if (n_rois > SHAPE3D_MAX_ROIS) return fail(SHAPE3D_EINVAL, "too many ROIs");
  if (dtype != SHAPE3D_U8 && dtype != SHAPE3D_F32) return fail(SHAPE3D_EINVAL, "bad dtype");
  const size_t elem = dtype == SHAPE3D_U8 ? 1 : 4;
  const char* abase;
  size_t asize;
  int rc = device_range(base, &abase, &asize);
  if (rc) return rc;
  for (int64_t r = 0; r < n_rois; ++r) {
    if ((rc = check_dims_spacing(rois[r].dims, rois[r].spacing))) return rc;
    if (rois[r].offset < 0) return fail(SHAPE3D_EINVAL, "negative ROI offset");
    const char* v = (const char*)base + (size_t)rois[r].offset * elem;
    const size_t need = (size_t)rois[r].dims[0] * (size_t)rois[r].dims[1] * (size_t)rois[r].dims[2] * elem;
    if (abase && v + need > abase + asize) return fail(SHAPE3D_EINVAL, "ROI extends past the end of the allocation");
    batch_add(Bt, v, rois[r].dims, rois[r].spacing);
    if (Bt.nbricks > (1ll << 31) - 1) return fail(SHAPE3D_EINVAL, "batch too large");
  }
  return SHAPE3D_OK;
}

int batched_impl(const void* base, int dtype, const shape3d_roi* rois, int64_t n_rois, int flags, hipStream_t st,
                 const RoiResult** hres_out) {
  Batch Bt;
  int rc = make_batch(base, dtype, rois, n_rois, Bt);
  if (rc) return rc;
  Workspace* wp = nullptr;
  if ((rc = get_workspace(&wp))) return rc;
  Workspace& w = *wp;
  if ((rc = ensure_layout_bufs(w, Bt))) return rc;
  const bool use_graph = (flags & SHAPE3D_BATCH_GRAPH) != 0;
  const std::string sig = use_graph ? layout_signature(base, dtype, rois, n_rois) : std::string();
  const RoiResult* hres = nullptr;
  bool done = false;
  if (use_graph) {
    auto it = w.graphs.find(sig);
    if (it != w.graphs.end() && it->second.generation == w.generation && it->second.exec) {
      // the ROI table of this layout is still on the device only if no other layout ran since
      char* h = (char*)w.host;
      memcpy(h + 4096, Bt.rois.data(), sizeof(Roi) * Bt.n());
      hipStream_t gs = w.graph_stream;
      HIPCK(hipEventRecord(w.ev[0], st));  // the caller's earlier work (e.g. writing the masks) first
      HIPCK(hipStreamWaitEvent(gs, w.ev[0], 0));
      HIPCK(hipMemcpyAsync(w.rois.p, h + 4096, sizeof(Roi) * Bt.n(), hipMemcpyHostToDevice, gs));
      HIPCK(hipGraphLaunch(it->second.exec, gs));
      HIPCK(hipStreamSynchronize(gs));
      hres = it->second.host_res;
      done = true;
      for (int64_t r = 0; r < n_rois; ++r)
        if (hres[r].status < 0) done = false;  // capacity exceeded on new contents: run eagerly
    }
  }
  if (done) w.graphs[sig].stamp = ++w.stamp;
  if (!done) {
    RoiResult* eager = host_results(w, Bt);
    if ((rc = run_eager(w, Bt, dtype, st, eager, 0, nullptr))) return rc;
    hres = eager;
    if (use_graph) {
      while (w.graphs.size() >= kMaxGraphs) {  // drop the least recently used graph
        auto lru = w.graphs.begin();
        for (auto g = w.graphs.begin(); g != w.graphs.end(); ++g)
          if (g->second.stamp < lru->second.stamp) lru = g;
        if (lru->second.exec) (void)hipGraphExecDestroy(lru->second.exec);
        if (lru->second.host_res) (void)hipHostFree(lru->second.host_res);
        w.graphs.erase(lru);
      }
      auto old = w.graphs.find(sig);
      if (old != w.graphs.end()) {
        if (old->second.exec) (void)hipGraphExecDestroy(old->second.exec);
        if (old->second.host_res) (void)hipHostFree(old->second.host_res);
        w.graphs.erase(old);
      }
      GraphRec rec;
      HIPCK(hipStreamSynchronize(st));
      rc = capture_graph(w, Bt, dtype, w.graph_stream, rec);
      if (rc) {
        if (rec.exec) (void)hipGraphExecDestroy(rec.exec);
        if (rec.host_res) (void)hipHostFree(rec.host_res);
        return rc;
      }
      rec.stamp = ++w.stamp;
      w.graphs.emplace(sig, rec);
    }
  }
  *hres_out = hres;
  for (int64_t r = 0; r < n_rois; ++r)
    if (hres[r].status < 0) return fail(hres[r].status, "an internal capacity was exceeded");
  return SHAPE3D_OK;
}

void fill_saved(shape3d_soft_saved* saved, const int64_t dims[3], const double spacing[3], const RoiResult& raw,
                int status) {
  for (int k = 0; k < 3; ++k) {
    saved->dims[k] = dims[k];
    saved->spacing[k] = spacing[k];
  }
  const bool empty = status == SHAPE3D_EMPTY;
  for (int f = 0; f < 6; ++f) saved->features[f] = empty ? 0.0 : raw.out[f];
  saved->signed_volume = empty ? 0.0 : raw.vol_signed;
  for (int f = 0; f < 4; ++f) {
    saved->pair_ids[f][0] = empty ? -1 : raw.ids[f][0];
    saved->pair_ids[f][1] = empty ? -1 : raw.ids[f][1];
  }
  saved->n_vertices = empty ? 0 : raw.V;
  saved->status = status;
}

// dL/dp of every ROI of a table (arguments already checked against their allocations).
int soft_backward_impl(const float* base, const shape3d_roi* rois, int64_t n_rois, const shape3d_soft_saved* saved,
                       const double* grad_out, float* grad_base, hipStream_t st) {
  int rc;
  Workspace* wp = nullptr;
  if ((rc = get_workspace(&wp))) return rc;
  Workspace& w = *wp;
  std::vector<SoftBwdRoi> table((size_t)n_rois);
  long long n_cblocks = 0, n_vblocks = 0, n_field = 0, cap = 0;
  for (int64_t r = 0; r < n_rois; ++r) {
    const shape3d_soft_saved& S = saved[r];
    for (int k = 0; k < 3; ++k)
      if (S.dims[k] != rois[r].dims[k] || S.spacing[k] != rois[r].spacing[k])
        return fail(SHAPE3D_EINVAL, "saved context does not match the ROI");
    if (S.status != SHAPE3D_OK && S.status != SHAPE3D_EMPTY) return fail(SHAPE3D_EINVAL, "saved context of a failed call");
    if (S.n_vertices < 0) return fail(SHAPE3D_EINVAL, "bad saved vertex count");
    for (int f = 0; f < 6; ++f)
      if (!std::isfinite(grad_out[6 * r + f])) return fail(SHAPE3D_EINVAL, "grad_out must be finite");
    SoftBwdRoi& R = table[(size_t)r];
    memset(&R, 0, sizeof(R));
    R.p = base + rois[r].offset;
    R.grad = grad_base + rois[r].offset;
    for (int k = 0; k < 3; ++k) {
      R.d[k] = (int)rois[r].dims[k];
      R.s[k] = rois[r].spacing[k];
      R.o[k] = 0.5 * (double)rois[r].dims[k] * rois[r].spacing[k];
    }
    const double* g = grad_out + 6 * r;
    R.g_area = g[1];
    R.g_vol_signed = g[0] * (S.signed_volume >= 0.0 ? 1.0 : -1.0);
    for (int f = 0; f < 4; ++f) {
      const double D = S.features[2 + f];
      const bool has = S.status == SHAPE3D_OK && D > 0.0 && S.pair_ids[f][0] >= 0 && S.pair_ids[f][1] >= 0;
      R.gdiam[f] = has ? g[2 + f] / D : 0.0;
      R.pair_ids[f][0] = S.pair_ids[f][0];
      R.pair_ids[f][1] = S.pair_ids[f][1];
    }
    const long long ncube = (long long)(R.d[0] + 1) * (R.d[1] + 1) * (R.d[2] + 1);
    const long long nvox = (long long)R.d[0] * R.d[1] * R.d[2];
    if (ncube >= (1ll << 31)) return fail(SHAPE3D_EINVAL, "soft ROI too large for the backward pass (2^31 cubes)");
    R.n_cubes = (unsigned int)ncube;
    R.n_vox = (unsigned int)nvox;
    magic_div((unsigned int)((R.d[1] + 1) * (R.d[2] + 1)), R.m_cplane, R.sh_cplane);
    magic_div((unsigned int)(R.d[2] + 1), R.m_c2, R.sh_c2);
    magic_div((unsigned int)(R.d[1] * R.d[2]), R.m_plane, R.sh_plane);
    magic_div((unsigned int)R.d[2], R.m_d2, R.sh_d2);
    R.field_begin = n_field;
    R.cblk_begin = n_cblocks;
    R.vblk_begin = n_vblocks;
    n_field += 3 * ncube;
    n_cblocks += (ncube + kCubeBlock - 1) / kCubeBlock;
    n_vblocks += (nvox + kVoxBlock - 1) / kVoxBlock;
    cap += S.n_vertices;
  }
  if (n_cblocks > (1ll << 31) - 2 || n_vblocks > (1ll << 31) - 2) return fail(SHAPE3D_EINVAL, "batch too large");
  const size_t tbytes = sizeof(SoftBwdRoi) * (size_t)n_rois;
  if ((rc = ensure(w, w.soft_rois, tbytes))) return rc;
  if ((rc = ensure(w, w.soft_edges, sizeof(unsigned long long) * std::max<long long>(cap, 1)))) return rc;
  // one float per grid edge; only crossing edges' slots are ever written or read
  if ((rc = ensure(w, w.soft_field, sizeof(float) * n_field))) return rc;
  if ((rc = ensure(w, w.soft_ctr, sizeof(long long) * 2))) return rc;
  // with more than a few ROIs, a table gives each workgroup its ROI (instead
  // of a binary search of the ROI table per workgroup)
  const bool blk_table = n_rois > 8;
  if (blk_table && (rc = ensure(w, w.soft_blk, sizeof(int) * (size_t)(n_cblocks + n_vblocks)))) return rc;
  if ((rc = ensure_host(w, std::max<size_t>(w.host_cap, 4096 + tbytes)))) return rc;
  char* h = (char*)w.host;
  memcpy(h + 4096, table.data(), tbytes);
  HIPCK(hipMemcpyAsync(w.soft_rois.p, h + 4096, tbytes, hipMemcpyHostToDevice, st));
  SoftBwdBufs B;
  B.rois = (const SoftBwdRoi*)w.soft_rois.p;
  B.n_rois = (int)n_rois;
  B.n_cblocks = n_cblocks;
  B.n_vblocks = n_vblocks;
  B.cap = cap;
  B.edges = (unsigned long long*)w.soft_edges.p;
  B.field = (float*)w.soft_field.p;
  B.n_field = n_field;
  B.counters = (long long*)w.soft_ctr.p;
  B.cu_count = w.cu_count;
  B.blk_roi = blk_table ? (int*)w.soft_blk.p : nullptr;
  HIPCK(launch_soft_backward(B, st));
  long long* used = (long long*)h;
  HIPCK(hipMemcpyAsync(used, w.soft_ctr.p, sizeof(long long), hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  if (*used != cap)
    return fail(SHAPE3D_EINVAL, "the probabilities differ from those of the forward pass (crossing edges " +
                                    std::to_string(*used) + ", saved " + std::to_string(cap) + "); grad is undefined");
  g_err.clear();
  return SHAPE3D_OK;
}

// Workload class of a batch for the tuning cache: dtype, and the binary
// orders of magnitude of the ROI count, of the total and of the largest
// vertex count (the pair work is about sum V^2 / 2).
std::string tuning_key(int dtype, int64_t n_rois, const RoiResult* res) {
  long long vsum = 0, vmax = 0;
  for (int64_t r = 0; r < n_rois; ++r) {
    vsum += res[r].V;
    vmax = std::max(vmax, res[r].V);
  }
  auto lg = [](long long x) { return x > 0 ? (int)std::lround(std::log2((double)x)) : -1; };
  char buf[96];
  snprintf(buf, sizeof(buf), "%s:n%d:v%d:m%d", dtype == SHAPE3D_U8 ? "u8" : "f32", lg(n_rois), lg(vsum), lg(vmax));
  return buf;
}

// Looks `key` up in a tuning cache file (lines "key kernel itile jchunk blocks_per_cu ms").
bool tuning_cache_find(const char* path, const std::string& key, Tuning& t, double& ms) {
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[256], k[128];
  bool found = false;
  while (fgets(line, sizeof(line), f)) {
    Tuning c;
    double m;
    if (sscanf(line, "%127s %d %d %d %d %lf", k, &c.kernel, &c.itile, &c.jchunk, &c.blocks_per_cu, &m) == 6 &&
        key == k && valid_tuning(c)) {
      t = c;  // the last entry for a key wins
      ms = m;
      found = true;
    }
  }
  fclose(f);
  return found;
}

int autotune_impl(const void* base, int dtype, const shape3d_roi* rois, int64_t n_rois, int reps,
                  const char* cache_path, Tuning& best, double& best_ms, hipStream_t st) {
  Batch Bt;
  int rc = make_batch(base, dtype, rois, n_rois, Bt);
  if (rc) return rc;
  if (reps < 1 || reps > 100) return fail(SHAPE3D_EINVAL, "reps must be in [1, 100]");
  Workspace* wp = nullptr;
  if ((rc = get_workspace(&wp))) return rc;
  Workspace& w = *wp;
  if ((rc = ensure_layout_bufs(w, Bt))) return rc;
  const Tuning saved = g_tune;
  // reference run with the current tiles: vertex counts (for the cache key) and results
  std::vector<RoiResult> ref((size_t)n_rois);
  RoiResult* hres = host_results(w, Bt);
  float ms[8] = {0};
  if ((rc = run_eager(w, Bt, dtype, st, hres, 1, ms))) return rc;
  for (int64_t r = 0; r < n_rois; ++r)
    if (hres[r].status < 0) return fail(hres[r].status, "an internal capacity was exceeded");
  std::copy(hres, hres + n_rois, ref.begin());
  const std::string key = tuning_key(dtype, n_rois, ref.data());
  if (cache_path && tuning_cache_find(cache_path, key, best, best_ms)) {
    g_tune = best;
    for (auto& kv : g_ws) drop_graphs(*kv.second);
    return SHAPE3D_OK;
  }
  best_ms = 1e300;
  best = saved;
  static const int kCand[5][2] = {{0, 2}, {0, 4}, {0, 8}, {1, 4}, {1, 8}};  // (kernel, itile)
  for (const auto& kc : kCand)
    for (int jc : {64, 128, 256, 512, 1024}) {
      g_tune = Tuning{kc[1], jc, 0, kc[0]};
      double t = 1e300;
      for (int k = 0; k < reps; ++k) {
        if ((rc = run_eager(w, Bt, dtype, st, hres, 1, ms))) {
          g_tune = saved;
          return rc;
        }
        t = std::min(t, (double)ms[3]);
      }
      // the tiles only change the work order: every result must be identical
      for (int64_t r = 0; r < n_rois; ++r)
        if (memcmp(hres[r].out, ref[(size_t)r].out, sizeof(ref[0].out)) != 0 ||
            memcmp(hres[r].ids, ref[(size_t)r].ids, sizeof(ref[0].ids)) != 0 || hres[r].status != ref[(size_t)r].status) {
          g_tune = saved;
          return fail(SHAPE3D_EINTERNAL, "pair-pass tiles changed a result");
        }
      if (t < best_ms) {
        best_ms = t;
        best = g_tune;
      }
    }
  g_tune = best;
  for (auto& kv : g_ws) drop_graphs(*kv.second);
  if (cache_path) {
    FILE* f = fopen(cache_path, "a");
    if (!f) return fail(SHAPE3D_EINVAL, std::string("cannot append to the tuning cache ") + cache_path);
    fprintf(f, "%s %d %d %d %d %.6f\n", key.c_str(), best.kernel, best.itile, best.jchunk, best.blocks_per_cu,
            best_ms);
    fclose(f);
  }
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

int shape3d_batched(const void* base, int dtype, const shape3d_roi* rois, int64_t n_rois, double* out, int* status,
                    int flags, void* stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!out || !status) return fail(SHAPE3D_EINVAL, "null output");
  const RoiResult* hres = nullptr;
  const int rc = batched_impl(base, dtype, rois, n_rois, flags, (hipStream_t)stream, &hres);
  if (rc < 0 && !hres) return rc;
  for (int64_t r = 0; r < n_rois; ++r) {
    for (int f = 0; f < 6; ++f) out[6 * r + f] = hres[r].out[f];
    status[r] = hres[r].status;
  }
  if (rc < 0) return rc;
  g_err.clear();
  return SHAPE3D_OK;
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
  Batch Bt;
  batch_add(Bt, vol, dims, spacing);
  if ((rc = ensure_layout_bufs(w, Bt))) return rc;
  char* h = (char*)w.host;
  memcpy(h + 4096, Bt.rois.data(), sizeof(Roi));
  HIPCK(hipMemcpyAsync(w.rois.p, h + 4096, sizeof(Roi), hipMemcpyHostToDevice, st));
  if ((rc = launch_head(w, Bt, dtype, st))) return rc;
  long long* th = (long long*)h;
  RoiMeta* mh = (RoiMeta*)(h + 1024);
  HIPCK(hipMemcpyAsync(th, w.totals.p, sizeof(long long) * 2, hipMemcpyDeviceToHost, st));
  HIPCK(hipMemcpyAsync(mh, w.meta.p, sizeof(RoiMeta), hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  const long long V = mh->V;
  *n_out = V;
  if (V > cap) return fail(SHAPE3D_ECAPACITY, "vertex buffer too small");
  if (V == 0) return SHAPE3D_EMPTY;
  Sizes S;
  if ((rc = ensure_vertex_bufs(w, Bt, dtype, th[0], S))) return rc;
  HIPCK(launch_check_capacity(1, S.rows0, (RoiMeta*)w.meta.p, (long long*)w.totals.p,
                              (unsigned int*)w.counters.p + 2, st));
  HIPCK(launch_mesh_emit(dtype, (const Roi*)w.rois.p, 1, Bt.nbricks, Bt.max_G, (const BrickPart*)w.part.p,
                         (const long long*)w.brick_voff.p, (const RoiMeta*)w.meta.p,
                         (const unsigned int*)w.counters.p + 2, (unsigned long long*)w.key.p,
                         dtype == SHAPE3D_F32 ? (double*)w.tsoft.p : nullptr, (float*)w.pos.p,
                         g_tune.kernel == 1 ? (uint4*)w.posh.p : nullptr, (int*)w.orig.p,
                         (int*)w.blkseg.p, (Seg*)w.segs.p, st));
  HIPCK(launch_export_vertices((const unsigned long long*)w.key.p,
                               dtype == SHAPE3D_F32 ? (const double*)w.tsoft.p : nullptr, (const RoiMeta*)w.meta.p,
                               (const Roi*)w.rois.p, (long long*)ids, pos, V, st));
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
  fill_saved(saved, dims, spacing, raw, rc);
  return rc;
}

int shape3d_soft_backward(const float* p, const shape3d_soft_saved* saved, const double grad_out[6], float* grad_p,
                          void* stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!saved || !grad_out || !grad_p) return fail(SHAPE3D_EINVAL, "null argument");
  shape3d_roi roi;
  roi.offset = 0;
  for (int k = 0; k < 3; ++k) {
    roi.dims[k] = saved->dims[k];
    roi.spacing[k] = saved->spacing[k];
  }
  int rc = check_args(p, SHAPE3D_F32, saved->dims, saved->spacing);
  if (!rc) rc = check_args(grad_p, SHAPE3D_F32, saved->dims, saved->spacing);
  if (rc) return rc;
  return soft_backward_impl(p, &roi, 1, saved, grad_out, grad_p, (hipStream_t)stream);
}

int shape3d_batched_soft_forward(const float* base, const shape3d_roi* rois, int64_t n_rois, double* out,
                                 shape3d_soft_saved* saved, int flags, void* stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!out || !saved) return fail(SHAPE3D_EINVAL, "null output");
  const RoiResult* hres = nullptr;
  const int rc = batched_impl(base, SHAPE3D_F32, rois, n_rois, flags, (hipStream_t)stream, &hres);
  if (rc < 0) return rc;
  for (int64_t r = 0; r < n_rois; ++r) {
    for (int f = 0; f < 6; ++f) out[6 * r + f] = hres[r].out[f];
    fill_saved(&saved[r], rois[r].dims, rois[r].spacing, hres[r], hres[r].status);
  }
  g_err.clear();
  return SHAPE3D_OK;
}

int shape3d_batched_soft_backward(const float* base, const shape3d_roi* rois, int64_t n_rois,
                                  const shape3d_soft_saved* saved, const double* grad_out, float* grad_base,
                                  void* stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!base || !rois || !saved || !grad_out || !grad_base || n_rois < 1)
    return fail(SHAPE3D_EINVAL, "null argument or empty batch");
  if (n_rois > SHAPE3D_MAX_ROIS) return fail(SHAPE3D_EINVAL, "too many ROIs");
  const char *pb, *gb;
  size_t ps, gs;
  int rc = device_range(base, &pb, &ps);
  if (!rc) rc = device_range(grad_base, &gb, &gs);
  if (rc) return rc;
  for (int64_t r = 0; r < n_rois; ++r) {
    if ((rc = check_dims_spacing(rois[r].dims, rois[r].spacing))) return rc;
    if (rois[r].offset < 0) return fail(SHAPE3D_EINVAL, "negative ROI offset");
    const size_t need = (size_t)rois[r].dims[0] * (size_t)rois[r].dims[1] * (size_t)rois[r].dims[2] * 4;
    const size_t off = (size_t)rois[r].offset * 4;
    if ((pb && (const char*)base + off + need > pb + ps) || (gb && (const char*)grad_base + off + need > gb + gs))
      return fail(SHAPE3D_EINVAL, "ROI extends past the end of the allocation");
  }
  return soft_backward_impl(base, rois, n_rois, saved, grad_out, grad_base, (hipStream_t)stream);
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
    drop_graphs(*w);
    if (w->graph_stream) (void)hipStreamDestroy(w->graph_stream);
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

int shape3d_get_tuning(shape3d_tuning* t) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!t) return fail(SHAPE3D_EINVAL, "null argument");
  t->itile_blocks = g_tune.itile;
  t->jchunk_blocks = g_tune.jchunk;
  t->blocks_per_cu = g_tune.blocks_per_cu;
  t->kernel = g_tune.kernel;
  return SHAPE3D_OK;
}

int shape3d_set_tuning(const shape3d_tuning* t) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!t) return fail(SHAPE3D_EINVAL, "null argument");
  const Tuning c{t->itile_blocks, t->jchunk_blocks, t->blocks_per_cu, t->kernel};
  if (!valid_tuning(c)) return fail(SHAPE3D_EINVAL, "unsupported tile sizes");
  g_tune = c;
  for (auto& kv : g_ws) drop_graphs(*kv.second);  // recorded graphs hold the old tiles
  g_err.clear();
  return SHAPE3D_OK;
}

int shape3d_autotune(const void* base, int dtype, const shape3d_roi* rois, int64_t n_rois, int reps,
                     const char* cache_path, shape3d_tuning* best, double* best_ms, void* stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!best || !best_ms) return fail(SHAPE3D_EINVAL, "null output");
  Tuning b;
  double ms = 0.0;
  const int rc = autotune_impl(base, dtype, rois, n_rois, reps, cache_path, b, ms, (hipStream_t)stream);
  if (rc < 0) return rc;
  best->itile_blocks = b.itile;
  best->jchunk_blocks = b.jchunk;
  best->blocks_per_cu = b.blocks_per_cu;
  best->kernel = b.kernel;
  *best_ms = ms;
  g_err.clear();
  return SHAPE3D_OK;
}

int shape3d_version(void) { return 103; }

}  // extern "C"
