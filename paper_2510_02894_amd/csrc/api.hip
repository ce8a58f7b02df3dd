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
#include <condition_variable>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/shape3d.h"
#include "s3d_launch.h"

using namespace s3d;

static_assert(sizeof(shape3d_roi_ex) == sizeof(RoiDesc), "shape3d_roi_ex and RoiDesc must have one layout");
static_assert(offsetof(shape3d_roi_ex, label) == offsetof(RoiDesc, label), "shape3d_roi_ex and RoiDesc must have one layout");

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

// Device buffers of the forward pipeline.  The layout buffers depend on the
// batch shape only (ROIs, bricks, plane buckets); the vertex buffers also on
// the layout-0 row capacity.  The library's own workspace grows each buffer
// on demand; a caller's workspace is carved into all of them at once.
enum WsId {
  W_ROIS, W_PLAN, W_PART, W_BRICK_VOFF, W_BRICK_ROI, W_META, W_CASE_AREA, W_TOTALS, W_COUNTERS, W_GRES, W_RES, W_PAIRS2D,
  W_BCNT, W_BCUR, W_BSZ, W_BFLAG, W_BROW, W_BSEG, W_BGROUP, W_BBOX,
  W_FIRST_VERTEX_BUF,
  W_KEY = W_FIRST_VERTEX_BUF, W_TSOFT, W_POS, W_POSH, W_ORIG, W_ROWMAX, W_BLKSEG, W_SEGS, W_NCOL, W_COLBASE,
  W_COLS, W_NITEM, W_ITEMBASE, W_SCAN_TMP, W_CAND, W_CAND_NCH, W_CAND_CHBASE, W_BLKREC, W_RSEED, W_PITEM,
  // the mesh pass's staging list (in the library's workspace sized on its own,
  // before the vertex count is known)
  W_TMPKEY, W_TMPT,
  W_NUM
};

struct Ptrs {
  void* p[W_NUM] = {};
  template <typename T>
  T* as(int i) const {
    return (T*)p[i];
  }
};

struct GraphRec {
  hipGraphExec_t exec = nullptr;
  long long generation = -1;
  RoiResult* host_res = nullptr;  // pinned, written by the graph's last copy (host-output graphs)
  long long n_rois = 0;
  long long stamp = 0;            // last use (the least recently used graph is dropped first)
};

constexpr size_t kMaxGraphs = 64;  // recorded batch layouts kept per device

struct Workspace {
  int device = -1;
  int cu_count = 0;
  long long generation = 0;  // bumped whenever a buffer is reallocated (graphs hold pointers)
  Buf buf[W_NUM];
  Buf soft_rois, soft_edges, soft_field, soft_ctr, soft_blk;  // soft backward
  void* host = nullptr;  // pinned staging: ROI table, read-backs, results
  size_t host_cap = 0;
  hipEvent_t ev[8] = {};
  bool events = false;
  hipStream_t graph_stream = nullptr;  // graphs are recorded and replayed here (the caller's
                                       // stream may be the legacy null stream, which cannot record)
  long long rows0_cap = 0;   // layout-0 rows the vertex buffers were sized for
  long long last_rows0 = 0;  // layout-0 rows of the last eager run (a recorded graph is sized for them)
  long long last_vmax = 0;   // largest vertex count of the last eager run
  std::map<std::string, GraphRec> graphs;
  long long stamp = 0;
  Buf small_slots;  // the small-mesh pair kernels' accumulators (SmallAcc)
  // host-to-device streaming (shape3d_host_stream): two device volumes, two
  // pinned chunks for pageable sources, the copy stream and its events
  Buf hs_vol[2];
  void* hs_pin[2] = {nullptr, nullptr};
  hipStream_t hs_copy = nullptr;
  hipEvent_t hs_ev[6] = {};  // 0, 1: a volume copied; 2, 3: a volume used; 4, 5: a pinned chunk free

  Ptrs ptrs() const {
    Ptrs P;
    for (int i = 0; i < W_NUM; ++i) P.p[i] = buf[i].p;
    return P;
  }
  std::vector<Buf*> soft_bufs() { return {&soft_rois, &soft_edges, &soft_field, &soft_ctr, &soft_blk}; }
};

std::map<int, Workspace*> g_ws;

// Scratch memory of shape3d_noalloc: one static device array per GPU (each
// device holds its own copy until the process ends).  Host code never uses the
// array's name as a device address: g_scratch[dev] holds the address that
// hipGetSymbolAddress returned for it on device dev.
constexpr int kMaxScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[SHAPE3D_NOALLOC_SCRATCH_BYTES];
void* g_scratch[kMaxScratchDevices] = {};

// Tile sizes of the pair pass for every device (results do not depend on them).
Tuning g_tune = {8, 1024, 0, 1, 1, 1};

// Vertex count from which a ROI's 3D pairs are pruned: kPruneMinV for prune = 1,
// every ROI with pairs for prune = 2.
int prune_min_v() { return g_tune.prune == 2 ? 2 : kPruneMinV; }

bool valid_tuning(const Tuning& t) {
  return (t.itile == 2 || t.itile == 4 || t.itile == 8) &&
         (t.jchunk == 64 || t.jchunk == 128 || t.jchunk == 256 || t.jchunk == 512 || t.jchunk == 1024) && t.blocks_per_cu >= 0 &&
         t.blocks_per_cu <= 64 && (t.kernel == 0 || (t.kernel == 1 && t.itile >= 4)) && (t.prune >= 0 && t.prune <= 2) &&
         (t.small_path == 0 || t.small_path == 1);
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

int device_cu_count(int dev, int* cu) {
  HIPCK(hipDeviceGetAttribute(cu, hipDeviceAttributeMultiprocessorCount, dev));
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
    int rc = device_cu_count(dev, &w->cu_count);
    if (rc) {
      delete w;
      return rc;
    }
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
int device_range(const void* ptr, const char** base, size_t* size, const char* what = "volume") {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, ptr) != hipSuccess) {
    (void)hipGetLastError();
    return fail(SHAPE3D_EINVAL, std::string(what) + " pointer is not HIP device memory");
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(SHAPE3D_EINVAL, std::string(what) + " pointer is not HIP device memory");
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

// Checks that [ptr, ptr + bytes) is device memory inside one allocation.
int check_device_span(const void* ptr, size_t bytes, const char* what) {
  if (!ptr) return fail(SHAPE3D_EINVAL, std::string("null ") + what);
  const char* base;
  size_t size;
  int rc = device_range(ptr, &base, &size, what);
  if (rc) return rc;
  if (base && (const char*)ptr + bytes > base + size)
    return fail(SHAPE3D_EINVAL, std::string(what) + " extends past the end of its allocation");
  return SHAPE3D_OK;
}

int check_args(const void* vol, int dtype, const int64_t dims[3], const double spacing[3]) {
  if (!vol || !dims || !spacing) return fail(SHAPE3D_EINVAL, "null argument");
  if (dtype != SHAPE3D_U8 && dtype != SHAPE3D_F32) return fail(SHAPE3D_EINVAL, "dtype must be SHAPE3D_U8 or SHAPE3D_F32");
  int rc = check_dims_spacing(dims, spacing);
  if (rc) return rc;
  const size_t need = (size_t)dims[0] * (size_t)dims[1] * (size_t)dims[2] * (dtype == SHAPE3D_U8 ? 1 : 4);
  return check_device_span(vol, need, "volume");
}

// Host description of a batch: its ROIs (host tables), or only bounds on its
// shape (tables planned on the device, `planned`).
struct Batch {
  std::vector<Roi> rois;
  int n_rois = 0;
  long long nbricks = 0;    // bricks (a bound when planned)
  long long n_buckets = 0;  // plane buckets (a bound when planned)
  int max_G = 1;
  bool planned = false;
  long long max_d[3] = {0, 0, 0};  // every ROI's dims are at most these
  bool moments = false;  // also the inside-voxel moments and the whole Shape class
  int n() const { return n_rois; }
  int nf() const { return moments ? SHAPE3D_N_CLASS : 6; }  // features per ROI in out
};

void batch_add(Batch& B, const void* vol, const int64_t dims[3], const double spacing[3], long long stride0 = 0,
               long long stride1 = 0, int label = 0, int tz = kTZ) {
  Roi R;
  memset(&R, 0, sizeof(R));
  const long long d[3] = {dims[0], dims[1], dims[2]};
  const long long nb = roi_fill(R, vol, d, spacing, stride0, stride1, label, tz);
  R.brick_begin = B.nbricks;
  R.brick_end = B.nbricks + nb;
  roi_set_buckets(R, B.n_buckets);
  B.nbricks += nb;
  B.n_buckets += roi_buckets(R.d);
  B.max_G = std::max(B.max_G, R.G);
  for (int k = 0; k < 3; ++k) B.max_d[k] = std::max(B.max_d[k], d[k]);
  B.rois.push_back(R);
  B.n_rois = (int)B.rois.size();
}

// Bounds of a batch of n ROIs planned on the device, each at most max_dims.
int batch_bounds(Batch& B, int64_t n, const int64_t max_dims[3]) {
  const double one[3] = {1.0, 1.0, 1.0};
  int rc = check_dims_spacing(max_dims, one);
  if (rc) return rc;
  Roi R;
  memset(&R, 0, sizeof(R));
  const long long d[3] = {max_dims[0], max_dims[1], max_dims[2]};
  const long long nb = roi_fill(R, nullptr, d, one, 0, 0, 0);
  B.planned = true;
  B.n_rois = (int)n;
  for (int k = 0; k < 3; ++k) B.max_d[k] = max_dims[k];
  B.nbricks = nb * n;
  B.n_buckets = roi_buckets(R.d) * n;
  B.max_G = R.G;
  if (B.nbricks > (1ll << 31) - 1) return fail(SHAPE3D_EINVAL, "batch too large (bricks of n_rois ROIs of max_dims)");
  return SHAPE3D_OK;
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

// Row indices of every layout are 32-bit in the kernels.
constexpr long long kMaxRows = (1ll << 31) - 1024;

// Byte sizes of every buffer for a batch and a layout-0 row capacity.
struct Layout {
  size_t bytes[W_NUM];
  Sizes S;
};

int ws_layout(const Batch& B, int dtype, const Tuning& t, long long rows0_cap, Layout& L) {
  const Sizes S = sizes_for(B, rows0_cap);
  if (S.rows_bound > kMaxRows || B.n_buckets > kMaxRows)
    return fail(SHAPE3D_ECAPACITY, "mesh too large: " + std::to_string(S.rows_bound) +
                                       " vertex rows exceed the 32-bit row indices of the kernels");
  const long long n = B.n();
  const long long scan_n = std::max(std::max(B.n_buckets, S.rows_bound), std::max(S.seg_cap, S.col_cap));
  size_t* b = L.bytes;
  b[W_ROIS] = sizeof(Roi) * n;
  b[W_PLAN] = sizeof(long long) * 4;
  b[W_PART] = sizeof(BrickPart) * B.nbricks;
  b[W_BRICK_VOFF] = sizeof(long long) * B.nbricks;
  b[W_BRICK_ROI] = B.n() > 1 ? sizeof(int) * B.nbricks : 0;
  b[W_META] = sizeof(RoiMeta) * n;
  b[W_CASE_AREA] = (sizeof(double) + sizeof(unsigned long long)) * 256 * n;  // areas, then counts
  b[W_TOTALS] = sizeof(long long) * 16;
  b[W_COUNTERS] = sizeof(unsigned int) * kCounterWords;
  b[W_GRES] = sizeof(GroupRes) * 4 * n;
  b[W_RES] = sizeof(RoiResult) * n;
  b[W_PAIRS2D] = sizeof(long long) * n;
  b[W_BCNT] = b[W_BCUR] = sizeof(unsigned int) * B.n_buckets;
  b[W_BSZ] = b[W_BFLAG] = b[W_BROW] = b[W_BSEG] = sizeof(long long) * B.n_buckets;
  b[W_BGROUP] = sizeof(int) * B.n_buckets;
  b[W_BBOX] = t.kernel == 1 ? sizeof(int) * 4 * B.n_buckets : 0;
  const long long r0 = std::max<long long>(S.rows0, 1);
  b[W_KEY] = sizeof(unsigned long long) * r0;
  b[W_TSOFT] = dtype == SHAPE3D_F32 ? sizeof(double) * r0 : 0;
  // pair-pass operands: FP32 position blocks (kernel 0, 16 B per row) or
  // split-f16 B operands (kernel 1, 1 KB per 32-row block)
  b[W_POS] = t.kernel == 0 ? sizeof(float) * 4 * S.rows_bound : 0;
  b[W_POSH] = t.kernel == 1 ? (size_t)1024 * ((S.rows_bound + 31) / 32) : 0;
  b[W_ORIG] = sizeof(int) * S.rows_bound;
  b[W_ROWMAX] = sizeof(float) * S.rows_bound;
  b[W_BLKSEG] = sizeof(int) * (S.rows_bound / kBlk + 1);
  b[W_SEGS] = sizeof(Seg) * S.seg_cap;
  b[W_NCOL] = b[W_COLBASE] = sizeof(long long) * S.seg_cap;
  b[W_COLS] = sizeof(Col) * S.col_cap;
  b[W_NITEM] = b[W_ITEMBASE] = sizeof(long long) * S.col_cap;
  b[W_SCAN_TMP] = sizeof(long long) * scan_tmp_elems(scan_n);
  // candidate rows of the exact refinement: every row could be one
  b[W_CAND] = sizeof(int) * S.rows_bound;
  b[W_CAND_NCH] = b[W_CAND_CHBASE] = sizeof(long long) * S.rows_bound;
  // 3D pruning: a record per 32-row block of layout 0, a seed record per ROI,
  // and pruned items (one per 8 rows; a longer list falls back to all pairs)
  b[W_BLKREC] = t.kernel == 1 ? sizeof(BlkRec) * (S.rows0 / 32 + 1) : 0;
  b[W_RSEED] = t.kernel == 1 ? sizeof(RoiSeed) * n : 0;
  b[W_PITEM] = t.kernel == 1 ? sizeof(PItem) * (S.rows0 / 8 + 64) : 0;
  b[W_TMPKEY] = sizeof(unsigned long long) * r0;
  b[W_TMPT] = dtype == SHAPE3D_F32 ? sizeof(double) * r0 : 0;
  L.S = S;
  return SHAPE3D_OK;
}

size_t aligned(size_t x) { return (x + 255) & ~(size_t)255; }

size_t ws_total(const Layout& L) {
  size_t t = 0;
  for (int i = 0; i < W_NUM; ++i) t += aligned(std::max<size_t>(L.bytes[i], 1));
  return t;
}

// The largest layout-0 row capacity (a multiple of kSegAlign) whose buffers
// fit in `bytes`; -1 if not even an empty mesh fits.
long long rows_cap_for(const Batch& B, int dtype, const Tuning& t, size_t bytes) {
  Layout L;
  if (ws_layout(B, dtype, t, 0, L) || ws_total(L) > bytes) return -1;
  long long lo = 0, hi = kMaxRows / 4 / kSegAlign;  // in units of kSegAlign rows
  while (lo < hi) {
    const long long mid = (lo + hi + 1) / 2;
    if (!ws_layout(B, dtype, t, mid * kSegAlign, L) && ws_total(L) <= bytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  g_err.clear();
  return lo * kSegAlign;
}

// Pointers of a caller's workspace block laid out for L (256-byte aligned).
int carve(const Layout& L, void* ws, size_t ws_bytes, Ptrs& P) {
  if (((uintptr_t)ws & 255u) != 0) return fail(SHAPE3D_EINVAL, "workspace must be 256-byte aligned");
  size_t off = 0;
  for (int i = 0; i < W_NUM; ++i) {
    P.p[i] = (char*)ws + off;
    off += aligned(std::max<size_t>(L.bytes[i], 1));
  }
  if (off > ws_bytes) return fail(SHAPE3D_ECAPACITY, "workspace too small");
  return SHAPE3D_OK;
}

// Grows the library's buffers [from, to) to the sizes of L.
int ensure_bufs(Workspace& w, const Layout& L, int from, int to) {
  for (int i = from; i < to; ++i) {
    const int rc = ensure(w, w.buf[i], L.bytes[i]);
    if (rc) return rc;
  }
  return SHAPE3D_OK;
}

// Buffers that depend only on the batch shape.
int ensure_layout_bufs(Workspace& w, const Batch& B, int dtype) {
  Layout L;
  int rc = ws_layout(B, dtype, g_tune, 0, L);
  if (!rc) rc = ensure_bufs(w, L, 0, W_FIRST_VERTEX_BUF);
  if (rc) return rc;
  // pinned staging: [0, 4096) read-backs, then the ROI table, then the results
  const size_t host_need = 4096 + sizeof(Roi) * (size_t)B.n() + 256 + sizeof(RoiResult) * (size_t)B.n();
  return ensure_host(w, host_need);
}

RoiResult* host_results(Workspace& w, const Batch& B) {
  const uintptr_t p = (uintptr_t)w.host + 4096 + sizeof(Roi) * (size_t)B.n();
  return (RoiResult*)((p + 255) & ~(uintptr_t)255);
}

// Grows the vertex buffers to hold rows0 layout-0 rows (they never shrink) and
// returns in S the sizes of this call's work, which follow rows0 itself.
int ensure_vertex_bufs(Workspace& w, const Batch& B, int dtype, long long rows0, Sizes& S_call) {
  Layout L, Lc;
  int rc = ws_layout(B, dtype, g_tune, rows0, Lc);
  if (!rc) rc = ws_layout(B, dtype, g_tune, std::max<long long>(rows0, w.rows0_cap), L);
  if (!rc) rc = ensure_bufs(w, L, W_FIRST_VERTEX_BUF, W_TMPKEY);
  if (rc) return rc;
  S_call = Lc.S;
  w.rows0_cap = L.S.rows0;
  return SHAPE3D_OK;
}

// The staging list of the mesh pass in the library's workspace: rows for at
// least `rows` vertices.  Returns its capacity in rows in *cap.
int ensure_staging(Workspace& w, int dtype, long long rows, long long* cap) {
  rows = std::max<long long>(rows, 1);
  int rc = ensure(w, w.buf[W_TMPKEY], sizeof(unsigned long long) * (size_t)rows);
  if (!rc && dtype == SHAPE3D_F32) rc = ensure(w, w.buf[W_TMPT], sizeof(double) * (size_t)rows);
  if (rc) return rc;
  long long c = (long long)(w.buf[W_TMPKEY].cap / sizeof(unsigned long long));
  if (dtype == SHAPE3D_F32) c = std::min<long long>(c, (long long)(w.buf[W_TMPT].cap / sizeof(double)));
  *cap = c;
  return SHAPE3D_OK;
}

// A first guess of a batch's vertex rows for the staging list (one per 16
// voxels, within [2^16, 2^26]); a mesh with more is counted by a first mesh
// pass and the pass runs again with a list of the right size.
long long staging_guess(const Batch& Bt) {
  double vox = 0.0;
  if (Bt.planned) {
    vox = (double)Bt.n() * (double)Bt.max_d[0] * (double)Bt.max_d[1] * (double)Bt.max_d[2];
  } else {
    for (const Roi& R : Bt.rois) vox += (double)R.d[0] * (double)R.d[1] * (double)R.d[2];
  }
  const double g = vox / 16.0 + 32.0 * Bt.n();
  return (long long)std::min(std::max(g, 65536.0), (double)(1ll << 26));
}

PairBufs pair_bufs(const Ptrs& P, const Batch& Bt, int dtype, const Sizes& S, int cu_count) {
  PairBufs B;
  B.rois = P.as<const Roi>(W_ROIS);
  B.n_rois = Bt.n();
  B.nbricks = Bt.nbricks;
  B.part = P.as<const BrickPart>(W_PART);
  B.brick_voff = P.as<const long long>(W_BRICK_VOFF);
  B.bmap = Bt.n() > 1 ? P.as<const int>(W_BRICK_ROI) : nullptr;
  {
    // plane keys a brick can touch: 2 tz + 3 along axis 0, at most 2 (256 + 2) + 1
    // along axis 1 (256 row-groups of at least one group per row) and
    // 2 (d2 + 1) + 1 along axis 2; smaller windows keep more workgroups per CU
    const long long w = (2ll * kTZ + 3) + (2ll * (kBrickThreads + 2) + 1) + (2ll * (Bt.max_d[2] + 1) + 1);
    B.brick_win = (int)std::min<long long>(2048, (w + 255) / 256 * 256);
  }
  B.meta = P.as<const RoiMeta>(W_META);
  B.key = P.as<const unsigned long long>(W_KEY);
  B.tsoft = dtype == SHAPE3D_F32 ? P.as<const double>(W_TSOFT) : nullptr;
  B.pos = P.as<float>(W_POS);
  B.posh = P.as<uint4>(W_POSH);
  B.orig = P.as<int>(W_ORIG);
  B.rowmax = P.as<float>(W_ROWMAX);
  B.blkseg = P.as<int>(W_BLKSEG);
  B.segs = P.as<Seg>(W_SEGS);
  B.rows0 = S.rows0;
  B.n_buckets = Bt.n_buckets;
  B.bcnt = P.as<unsigned int>(W_BCNT);
  B.bcur = P.as<unsigned int>(W_BCUR);
  B.bsz = P.as<long long>(W_BSZ);
  B.bflag = P.as<long long>(W_BFLAG);
  B.bgroup = P.as<int>(W_BGROUP);
  B.brow = P.as<long long>(W_BROW);
  B.bseg = P.as<long long>(W_BSEG);
  B.bbox = P.as<int4>(W_BBOX);
  B.seg_cap = S.seg_cap;
  B.ncol = P.as<long long>(W_NCOL);
  B.colbase = P.as<long long>(W_COLBASE);
  B.col_cap = S.col_cap;
  B.cols = P.as<Col>(W_COLS);
  B.nitem = P.as<long long>(W_NITEM);
  B.itembase = P.as<long long>(W_ITEMBASE);
  B.totals = P.as<long long>(W_TOTALS);
  B.scan_tmp = P.as<long long>(W_SCAN_TMP);
  B.counters = P.as<unsigned int>(W_COUNTERS);
  B.gres = P.as<GroupRes>(W_GRES);
  B.cand = P.as<int>(W_CAND);
  B.cand_cap = S.rows_bound;
  B.tune = g_tune;
  B.max_rows_seg = S.rows0;
  B.rows_bound = S.rows_bound;
  B.res = P.as<RoiResult>(W_RES);
  B.pairs2d = P.as<long long>(W_PAIRS2D);
  B.cand_nch = P.as<long long>(W_CAND_NCH);
  B.cand_chbase = P.as<long long>(W_CAND_CHBASE);
  B.cu_count = cu_count;
  B.moments = Bt.moments;
  // canonical ids 3 lin(u) + a, lin over the padded (d + 2)^3 grid
  B.ids32 = 3.0 * (double)(Bt.max_d[0] + 2) * (double)(Bt.max_d[1] + 2) * (double)(Bt.max_d[2] + 2) < 4294967295.0;
  B.prune = false;
  B.prune_min_v = prune_min_v();
  B.blkrec = P.as<BlkRec>(W_BLKREC);
  B.rseed = P.as<RoiSeed>(W_RSEED);
  B.pitems = P.as<PItem>(W_PITEM);
  B.pitem_cap = S.rows0 / 8 + 64;
  return B;
}

// The mesh pass (with the staging list's capacity in rows) and per-ROI
// totals (launches only).
int launch_head(const Ptrs& P, const Batch& Bt, int dtype, long long tmp_cap, hipStream_t st) {
  HIPCK(launch_mesh_pass(dtype, P.as<const Roi>(W_ROIS), Bt.n(), Bt.nbricks, Bt.max_G, P.as<double>(W_CASE_AREA),
                         P.as<BrickPart>(W_PART), P.as<unsigned int>(W_COUNTERS), kCounterWords,
                         P.as<unsigned long long>(W_TMPKEY), dtype == SHAPE3D_F32 ? P.as<double>(W_TMPT) : nullptr,
                         tmp_cap, P.as<long long>(W_TOTALS), Bt.moments ? 1 : 0, P.as<int>(W_BRICK_ROI), st));
  HIPCK(launch_mesh_totals(P.as<const Roi>(W_ROIS), Bt.n(), Bt.nbricks, dtype, P.as<const double>(W_CASE_AREA),
                           P.as<const BrickPart>(W_PART),
                           P.as<long long>(W_BRICK_VOFF), P.as<RoiMeta>(W_META), P.as<long long>(W_TOTALS),
                           Bt.moments ? 1 : 0, prune_min_v(), st));
  return SHAPE3D_OK;
}

// The capacity check and layout 0 from the staging list of tmp_cap rows (launches only).
int launch_rows(const Ptrs& P, const Batch& Bt, int dtype, long long rows0_cap, long long tmp_cap, uint4* posh,
                hipStream_t st) {
  HIPCK(launch_mesh_rows(P.as<const Roi>(W_ROIS), Bt.n(), Bt.nbricks, P.as<const BrickPart>(W_PART),
                         P.as<const long long>(W_BRICK_VOFF), P.as<RoiMeta>(W_META), P.as<long long>(W_TOTALS),
                         rows0_cap, P.as<const unsigned long long>(W_TMPKEY),
                         dtype == SHAPE3D_F32 ? P.as<const double>(W_TMPT) : nullptr, tmp_cap,
                         P.as<unsigned long long>(W_KEY), dtype == SHAPE3D_F32 ? P.as<double>(W_TSOFT) : nullptr,
                         posh ? nullptr : P.as<float>(W_POS), posh, P.as<int>(W_ORIG), P.as<int>(W_BLKSEG),
                         P.as<Seg>(W_SEGS), P.as<unsigned int>(W_COUNTERS) + 2, P.as<const int>(W_BRICK_ROI), st));
  return SHAPE3D_OK;
}

// Everything after the totals, up to the per-ROI results in W_RES (launches
// only).  ev: optional phase events recorded before emission, buckets, pairs,
// refinement and finalisation.
// vmax_hint: the largest vertex count of the batch (a bound), or -1 if unknown;
// with prune = 1 the call prunes when it may reach kPruneCallMinV (then every
// ROI of at least kPruneMinV vertices), with prune = 2 always (every ROI).
int launch_tail(const Ptrs& P, const Batch& Bt, int dtype, const Sizes& S, long long tmp_cap, int cu_count,
                hipStream_t st, hipEvent_t* ev, long long vmax_hint) {
  PairBufs B = pair_bufs(P, Bt, dtype, S, cu_count);
  B.prune = g_tune.kernel == 1 &&
            (g_tune.prune == 2 || (g_tune.prune == 1 && (vmax_hint < 0 || vmax_hint >= kPruneCallMinV)));
  B.prune_min_v = prune_min_v();
  if (ev) HIPCK(hipEventRecord(ev[0], st));
  int rc = launch_rows(P, Bt, dtype, S.rows0, tmp_cap, split_rows(B), st);
  if (rc) return rc;
  if (ev) HIPCK(hipEventRecord(ev[1], st));
  if (B.prune) HIPCK(launch_prune(B, st));
  HIPCK(launch_buckets(B, st));
  HIPCK(launch_init_groups(B, st));  // also zeroes the row maxima
  if (ev) HIPCK(hipEventRecord(ev[2], st));
  HIPCK(launch_pair_maxima(B, st));
  if (ev) HIPCK(hipEventRecord(ev[3], st));
  HIPCK(launch_refine(B, st));
  if (ev) HIPCK(hipEventRecord(ev[4], st));
  HIPCK(launch_finalize(B, st));
  return SHAPE3D_OK;
}

// The ROI table into W_ROIS: a host table through the pinned staging buffer
// (library workspace), or planned on the device from a caller's descriptors.
struct DevTable {
  const RoiDesc* rois = nullptr;
  long long max_dims[3] = {0, 0, 0};
  const void* base = nullptr;
  long long alloc_elems = 0;
};

int upload_rois(Workspace& w, const Ptrs& P, const Batch& Bt, int dtype, const DevTable* dt, hipStream_t st) {
  if (dt) {
    HIPCK(launch_plan_rois(dt->rois, Bt.n(), dtype, dt->max_dims, dt->base, dt->alloc_elems, P.as<Roi>(W_ROIS),
                           P.as<long long>(W_PLAN), st));
    return SHAPE3D_OK;
  }
  char* h = (char*)w.host;
  memcpy(h + 4096, Bt.rois.data(), sizeof(Roi) * Bt.n());
  HIPCK(hipMemcpyAsync(P.p[W_ROIS], h + 4096, sizeof(Roi) * Bt.n(), hipMemcpyHostToDevice, st));
  return SHAPE3D_OK;
}

// One eager run of a batch on the library workspace; the per-ROI results are
// left in W_RES and, if host_res is set, copied there (pinned).
int run_eager(Workspace& w, const Batch& Bt, int dtype, hipStream_t st, RoiResult* host_res, int timing,
              float* phase_ms, const DevTable* dt = nullptr) {
  int rc;
  char* h = (char*)w.host;
  long long tcap = 0;
  if ((rc = ensure_staging(w, dtype, staging_guess(Bt), &tcap))) return rc;
  Ptrs P = w.ptrs();
  if ((rc = upload_rois(w, P, Bt, dtype, dt, st))) return rc;
  long long* th = (long long*)h;
  for (int pass = 0;; ++pass) {
    if (timing) HIPCK(hipEventRecord(w.ev[0], st));
    if ((rc = launch_head(P, Bt, dtype, tcap, st))) return rc;
    if (timing) HIPCK(hipEventRecord(w.ev[1], st));
    HIPCK(hipMemcpyAsync(th, P.p[W_TOTALS], sizeof(long long) * 9, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    if (th[8] <= tcap || pass > 0) break;
    // more vertices than the staging list held: size it and run the mesh pass again
    if ((rc = ensure_staging(w, dtype, th[8], &tcap))) return rc;
    P = w.ptrs();
  }
  if (th[8] > tcap) return fail(SHAPE3D_EINTERNAL, "the mesh pass's staging list overflowed twice");
  Sizes S;
  if ((rc = ensure_vertex_bufs(w, Bt, dtype, th[0], S))) return rc;
  P = w.ptrs();
  w.last_rows0 = th[0];
  w.last_vmax = th[1];
  if ((rc = launch_tail(P, Bt, dtype, S, tcap, w.cu_count, st, timing ? &w.ev[2] : nullptr, th[1]))) return rc;
  if (host_res) HIPCK(hipMemcpyAsync(host_res, P.p[W_RES], sizeof(RoiResult) * Bt.n(), hipMemcpyDeviceToHost, st));
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

// The whole pipeline on fixed buffers (a caller's workspace), without any
// host synchronisation: the ROI table is set on the device, the vertex
// capacity comes from the workspace size, and a mesh beyond it ends with
// status SHAPE3D_ECAPACITY for every ROI.  Results go to out/status (device).
int run_fixed(const Batch& Bt, int dtype, const Roi* one_roi, const DevTable* dt, void* ws, size_t ws_bytes,
              int cu_count, double* out, int* status, hipStream_t st) {
  const long long cap = rows_cap_for(Bt, dtype, g_tune, ws_bytes);
  if (cap < 0) return fail(SHAPE3D_ECAPACITY, "workspace too small for this input's mesh-pass buffers");
  Layout L;
  int rc = ws_layout(Bt, dtype, g_tune, cap, L);
  Ptrs P;
  if (!rc) rc = carve(L, ws, ws_bytes, P);
  if (rc) return rc;
  if (dt) {
    HIPCK(launch_plan_rois(dt->rois, Bt.n(), dtype, dt->max_dims, dt->base, dt->alloc_elems, P.as<Roi>(W_ROIS),
                           P.as<long long>(W_PLAN), st));
  } else {
    HIPCK(launch_set_roi(*one_roi, P.as<Roi>(W_ROIS), st));
  }
  if ((rc = launch_head(P, Bt, dtype, cap, st))) return rc;
  if ((rc = launch_tail(P, Bt, dtype, L.S, cap, cu_count, st, nullptr, cap))) return rc;
  HIPCK(launch_results_out(P.as<const RoiResult>(W_RES), Bt.n(), out, status, Bt.nf(), st));
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

// The small-mesh path of one ROI: the ROI record, the mesh pass into the
// staging list and the exact all-pairs kernel (three launches), then the
// result read back.  hres->status is kSmallOverflow when the mesh has more
// than kSmallMaxV vertices (the general path must run instead).
int run_small(Workspace& w, const void* vol, int dtype, const int64_t dims[3], const double spacing[3], hipStream_t st,
              RoiResult* hres) {
  // Binary masks: bricks of one cube plane, so that a small ROI still spreads
  // over many workgroups (the area is summed from per-case counts, whatever
  // the bricks).  Soft masks keep the general path's bricks: their area and
  // volume partials are summed per brick, and the results must not change.
  Batch Bt;
  batch_add(Bt, vol, dims, spacing, 0, 0, 0, dtype == SHAPE3D_U8 ? 1 : kTZ);
  int rc = ensure_layout_bufs(w, Bt, dtype);
  if (rc) return rc;
  long long tcap = 0;
  if ((rc = ensure_staging(w, dtype, kSmallMaxV, &tcap))) return rc;
  const int groups = 4 * w.cu_count;
  if ((rc = ensure(w, w.small_slots, small_acc_bytes()))) return rc;
  const Ptrs P = w.ptrs();
  SmallAcc* acc = (SmallAcc*)w.small_slots.p;
  const long long vmax = std::min(tcap, kSmallMaxV);
  HIPCK(launch_small_head(dtype, Bt.rois[0], P.as<Roi>(W_ROIS), P.as<long long>(W_TOTALS), acc,
                          P.as<double>(W_CASE_AREA), st));
  HIPCK(launch_mesh_core(dtype, P.as<const Roi>(W_ROIS), 1, Bt.nbricks, Bt.max_G, P.as<double>(W_CASE_AREA),
                         P.as<BrickPart>(W_PART), P.as<unsigned long long>(W_TMPKEY),
                         dtype == SHAPE3D_F32 ? P.as<double>(W_TMPT) : nullptr, vmax, P.as<long long>(W_TOTALS), 0,
                         st));
  HIPCK(launch_small_pairs(dtype, P.as<const Roi>(W_ROIS), P.as<const BrickPart>(W_PART), Bt.nbricks,
                           P.as<const double>(W_CASE_AREA), P.as<const unsigned long long>(W_TMPKEY),
                           dtype == SHAPE3D_F32 ? P.as<const double>(W_TMPT) : nullptr,
                           P.as<const long long>(W_TOTALS), vmax, acc, groups, P.as<RoiResult>(W_RES), st));
  HIPCK(hipMemcpyAsync(hres, P.p[W_RES], sizeof(RoiResult), hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  return SHAPE3D_OK;
}

// Whether a single-ROI call tries the small-mesh path first: six features,
// no phase timing, a ROI small enough that a mesh beyond kSmallMaxV vertices
// is unlikely (one that has more costs one extra mesh pass), and the
// tuning's small-path switch on.
bool small_path(const Batch& Bt, bool moments, int timing) {
  if (moments || timing || !g_tune.small_path || Bt.n() != 1) return false;
  const Roi& R = Bt.rois[0];
  // the pair kernels pack two canonical ids, below 3 (d0 + 2) (d1 + 2) (d2 + 2), in 64 bits
  const long long ids = 3ll * (R.d[0] + 2) * (R.d[1] + 2) * (R.d[2] + 2);
  return (long long)R.d[0] * R.d[1] * R.d[2] <= kSmallMaxVoxels && ids < (1ll << 32);
}

// out: the six features, or with `moments` the SHAPE3D_N_CLASS Shape-class members.
int shape3d_impl(const void* vol, int dtype, const int64_t dims[3], const double spacing[3], double* out,
                 shape3d_stats* stats, int timing, hipStream_t st, RoiResult* raw = nullptr, bool moments = false) {
  int rc = check_args(vol, dtype, dims, spacing);
  if (rc) return rc;
  if (!out) return fail(SHAPE3D_EINVAL, "null out");
  Workspace* wp = nullptr;
  if ((rc = get_workspace(&wp))) return rc;
  Workspace& w = *wp;
  Batch Bt;
  Bt.moments = moments;
  batch_add(Bt, vol, dims, spacing);
  if ((rc = ensure_layout_bufs(w, Bt, dtype))) return rc;
  RoiResult* hres = host_results(w, Bt);
  float ms[8] = {0};
  bool done = false;
  if (!raw && small_path(Bt, moments, timing)) {
    if ((rc = run_small(w, vol, dtype, dims, spacing, st, hres))) return rc;
    done = hres->status != kSmallOverflow;
  }
  if (!done && (rc = run_eager(w, Bt, dtype, st, hres, timing, ms))) return rc;
  if (hres->status < 0) return fail(hres->status, "an internal capacity was exceeded");
  for (int f = 0; f < 6; ++f) out[f] = hres->out[f];
  if (moments)
    for (int f = 6; f < SHAPE3D_N_CLASS; ++f) out[f] = hres->shape[f - 6];
  if (raw) *raw = *hres;
  fill_stats(stats, *hres, timing ? ms : nullptr);
  g_err.clear();
  return hres->status;
}

std::string layout_signature(const void* base, int dtype, const void* table, size_t table_bytes,
                             const void* extra = nullptr, size_t extra_bytes = 0) {
  std::string sig((const char*)&base, sizeof(base));
  sig.append((const char*)&dtype, sizeof(dtype));
  sig.append((const char*)table, table_bytes);
  if (extra) sig.append((const char*)extra, extra_bytes);
  return sig;
}

// Records the pipeline of a batch as a graph (buffers already sized by the
// eager run just made: a replay that finds more rows than that is caught by
// the capacity check).  Host tables: the ROI table is uploaded before each
// replay and the results are copied to rec.host_res.  Device tables
// (dt set): the graph plans the ROI table itself and ends with the results
// in out/status on the device.
int capture_graph(Workspace& w, const Batch& Bt, int dtype, hipStream_t st, GraphRec& rec,
                  const DevTable* dt = nullptr, double* out = nullptr, int* status = nullptr) {
  rec.n_rois = Bt.n();
  if (!dt) {
    if (hipHostMalloc((void**)&rec.host_res, sizeof(RoiResult) * Bt.n(), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      rec.host_res = nullptr;
      return fail(SHAPE3D_ENOMEM, "pinned host allocation failed");
    }
  }
  const Sizes S = sizes_for(Bt, w.last_rows0);
  // a staging list that holds the recorded row capacity, so that a replay
  // within that capacity stages every vertex
  long long tcap = 0;
  int rc0 = ensure_staging(w, dtype, w.last_rows0, &tcap);
  if (rc0) return rc0;
  const Ptrs P = w.ptrs();
  hipGraph_t graph = nullptr;
  HIPCK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  int rc = SHAPE3D_OK;
  if (dt) {
    const hipError_t e = launch_plan_rois(dt->rois, Bt.n(), dtype, dt->max_dims, dt->base, dt->alloc_elems,
                                          P.as<Roi>(W_ROIS), P.as<long long>(W_PLAN), st);
    if (e != hipSuccess) rc = fail(SHAPE3D_EHIP, std::string("plan: ") + hipGetErrorString(e));
  }
  if (!rc) rc = launch_head(P, Bt, dtype, tcap, st);
  if (!rc) rc = launch_tail(P, Bt, dtype, S, tcap, w.cu_count, st, nullptr, w.last_vmax);
  if (!rc) {
    const hipError_t e = dt ? launch_results_out(P.as<const RoiResult>(W_RES), Bt.n(), out, status, Bt.nf(), st)
                            : hipMemcpyAsync(rec.host_res, P.p[W_RES], sizeof(RoiResult) * Bt.n(),
                                             hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) rc = fail(SHAPE3D_EHIP, std::string("results: ") + hipGetErrorString(e));
  }
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

void erase_graph(Workspace& w, std::map<std::string, GraphRec>::iterator it) {
  if (it->second.exec) (void)hipGraphExecDestroy(it->second.exec);
  if (it->second.host_res) (void)hipHostFree(it->second.host_res);
  w.graphs.erase(it);
}

// Makes room for a new graph under `sig` (drops the least recently used ones
// and any old graph of the same signature).
void graph_slot(Workspace& w, const std::string& sig) {
  auto old = w.graphs.find(sig);
  if (old != w.graphs.end()) erase_graph(w, old);
  while (w.graphs.size() >= kMaxGraphs) {
    auto lru = w.graphs.begin();
    for (auto g = w.graphs.begin(); g != w.graphs.end(); ++g)
      if (g->second.stamp < lru->second.stamp) lru = g;
    erase_graph(w, lru);
  }
}

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

// The batched forward pass; on success *hres_out points at the per-ROI results
// (pinned host memory owned by the workspace, valid until the next call).
int batched_impl(const void* base, int dtype, const shape3d_roi* rois, int64_t n_rois, int flags, hipStream_t st,
                 const RoiResult** hres_out) {
  Batch Bt;
  Bt.moments = (flags & SHAPE3D_SHAPE_CLASS) != 0;
  int rc = make_batch(base, dtype, rois, n_rois, Bt);
  if (rc) return rc;
  Workspace* wp = nullptr;
  if ((rc = get_workspace(&wp))) return rc;
  Workspace& w = *wp;
  if ((rc = ensure_layout_bufs(w, Bt, dtype))) return rc;
  const bool use_graph = (flags & SHAPE3D_BATCH_GRAPH) != 0;
  const int sig_flags = flags & SHAPE3D_SHAPE_CLASS;
  const std::string sig = use_graph ? layout_signature(base, dtype, rois, sizeof(shape3d_roi) * (size_t)n_rois,
                                                       &sig_flags, sizeof(sig_flags))
                                    : std::string();
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
      HIPCK(hipMemcpyAsync(w.buf[W_ROIS].p, h + 4096, sizeof(Roi) * Bt.n(), hipMemcpyHostToDevice, gs));
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
      graph_slot(w, sig);
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

// The batched forward pass on a ROI table in device memory, with results left
// on the device (see shape3d_batched_dev).
int batched_dev_impl(const void* base, int dtype, const shape3d_roi_ex* rois, int64_t n_rois,
                     const int64_t max_dims[3], double* out, int* status, void* ws, size_t ws_bytes, int flags,
                     hipStream_t st) {
  if (!base || !rois || !max_dims || !out || !status || n_rois < 1)
    return fail(SHAPE3D_EINVAL, "null argument or empty batch");
  if (n_rois > SHAPE3D_MAX_ROIS) return fail(SHAPE3D_EINVAL, "too many ROIs");
  if (dtype != SHAPE3D_U8 && dtype != SHAPE3D_F32) return fail(SHAPE3D_EINVAL, "bad dtype");
  Batch Bt;
  int rc = batch_bounds(Bt, n_rois, max_dims);
  if (rc) return rc;
  Bt.moments = (flags & SHAPE3D_SHAPE_CLASS) != 0;
  const char* abase;
  size_t asize;
  if ((rc = device_range(base, &abase, &asize))) return rc;
  if (!abase) return fail(SHAPE3D_EINVAL, "the allocation holding base is unknown to the runtime");
  const size_t elem = dtype == SHAPE3D_U8 ? 1 : 4;
  if ((uintptr_t)base % elem) return fail(SHAPE3D_EINVAL, "misaligned base");
  if ((rc = check_device_span(rois, sizeof(shape3d_roi_ex) * (size_t)n_rois, "ROI table"))) return rc;
  if ((rc = check_device_span(out, sizeof(double) * Bt.nf() * (size_t)n_rois, "out"))) return rc;
  if ((rc = check_device_span(status, sizeof(int) * (size_t)n_rois, "status"))) return rc;
  DevTable dt;
  dt.rois = (const RoiDesc*)rois;
  for (int k = 0; k < 3; ++k) dt.max_dims[k] = max_dims[k];
  dt.base = base;
  dt.alloc_elems = (long long)(((size_t)(abase + asize - (const char*)base)) / elem);
  if (ws) {
    int dev = 0, cu = 0;
    HIPCK(hipGetDevice(&dev));
    if ((rc = device_cu_count(dev, &cu))) return rc;
    if ((rc = check_device_span(ws, ws_bytes, "workspace"))) return rc;
    return run_fixed(Bt, dtype, nullptr, &dt, ws, ws_bytes, cu, out, status, st);
  }
  Workspace* wp = nullptr;
  if ((rc = get_workspace(&wp))) return rc;
  Workspace& w = *wp;
  if ((rc = ensure_layout_bufs(w, Bt, dtype))) return rc;
  const bool use_graph = (flags & SHAPE3D_BATCH_GRAPH) != 0;
  std::string sig;
  if (use_graph) {
    const void* extra[3] = {rois, out, status};
    sig = layout_signature(base, dtype, max_dims, sizeof(int64_t) * 3, extra, sizeof(extra));
    sig.append((const char*)&n_rois, sizeof(n_rois));
    const int sig_flags = flags & SHAPE3D_SHAPE_CLASS;
    sig.append((const char*)&sig_flags, sizeof(sig_flags));
    auto it = w.graphs.find(sig);
    if (it != w.graphs.end() && it->second.generation == w.generation && it->second.exec) {
      hipStream_t gs = w.graph_stream;
      HIPCK(hipEventRecord(w.ev[0], st));  // the caller's earlier work (the table, the masks) first
      HIPCK(hipStreamWaitEvent(gs, w.ev[0], 0));
      HIPCK(hipGraphLaunch(it->second.exec, gs));
      HIPCK(hipEventRecord(w.ev[1], gs));  // and the caller's later work after the results
      HIPCK(hipStreamWaitEvent(st, w.ev[1], 0));
      it->second.stamp = ++w.stamp;
      g_err.clear();
      return SHAPE3D_OK;
    }
  }
  if ((rc = run_eager(w, Bt, dtype, st, nullptr, 0, nullptr, &dt))) return rc;
  HIPCK(launch_results_out(w.ptrs().as<const RoiResult>(W_RES), Bt.n(), out, status, Bt.nf(), st));
  if (use_graph) {
    graph_slot(w, sig);
    GraphRec rec;
    HIPCK(hipStreamSynchronize(st));
    rc = capture_graph(w, Bt, dtype, w.graph_stream, rec, &dt, out, status);
    if (rc) {
      if (rec.exec) (void)hipGraphExecDestroy(rec.exec);
      return rc;
    }
    rec.stamp = ++w.stamp;
    w.graphs.emplace(sig, rec);
  }
  g_err.clear();
  return SHAPE3D_OK;
}

// Bytes of a caller workspace for a batch shape and a bound on the vertex
// count (or the worst case of its dims when max_vertices < 0).
int workspace_size_impl(const Batch& Bt, int dtype, long long max_vertices, size_t* bytes) {
  if (!bytes) return fail(SHAPE3D_EINVAL, "null output");
  if (dtype != SHAPE3D_U8 && dtype != SHAPE3D_F32) return fail(SHAPE3D_EINVAL, "bad dtype");
  long long rows0;
  if (max_vertices < 0) {
    // every grid edge of every ROI's padded cube grid could cross
    long long worst = 0;
    if (Bt.planned) {
      worst = (3ll * (Bt.max_d[0] + 1) * (Bt.max_d[1] + 1) * (Bt.max_d[2] + 1) + kSegAlign) * Bt.n();
    } else {
      for (const Roi& R : Bt.rois) worst += 3ll * (R.d[0] + 1) * (R.d[1] + 1) * (R.d[2] + 1) + kSegAlign;
    }
    rows0 = worst;
  } else {
    rows0 = max_vertices + (long long)kSegAlign * Bt.n();
  }
  rows0 = (rows0 + kSegAlign - 1) / kSegAlign * kSegAlign;
  Layout L;
  const int rc = ws_layout(Bt, dtype, g_tune, std::min(rows0, kMaxRows), L);
  if (rc) return rc;
  if (rows0 > kMaxRows) return ws_layout(Bt, dtype, g_tune, rows0, L);
  *bytes = ws_total(L);
  g_err.clear();
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
    Tuning c = g_tune;  // the cache holds the tiles; pruning and the small path stay as set
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
  if ((rc = ensure_layout_bufs(w, Bt, dtype))) return rc;
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
      g_tune = Tuning{kc[1], jc, 0, kc[0], saved.prune, saved.small_path};
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

// ---------------------------------------------------------------------------
// Volumes that start in host memory (shape3d_host_stream).  A staging thread
// copies volume i + 1 to the device on its own stream while the calling
// thread computes volume i on the caller's stream; two device volumes
// alternate.  Page-locked sources go to the device in one DMA copy; pageable
// ones pass through two pinned chunks that alternate, so the host copy of one
// chunk overlaps the DMA of the other.

constexpr size_t kStreamChunk = 32ull << 20;

int host_stream_buffers(Workspace& w, size_t vol_bytes, bool pageable) {
  if (!w.hs_copy) {
    HIPCK(hipStreamCreateWithFlags(&w.hs_copy, hipStreamNonBlocking));
    for (hipEvent_t& e : w.hs_ev) HIPCK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  for (int i = 0; i < 2; ++i) {
    Buf& b = w.hs_vol[i];
    if (b.cap < vol_bytes) {
      HIPCK(hipDeviceSynchronize());
      if (b.p) (void)hipFree(b.p);
      b.p = nullptr;
      b.cap = 0;
      const size_t want = (vol_bytes + 255) & ~(size_t)255;
      if (hipMalloc(&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(SHAPE3D_ENOMEM, "device allocation of a staging volume failed");
      }
      b.cap = want;
    }
    if (pageable && !w.hs_pin[i]) {
      if (hipHostMalloc(&w.hs_pin[i], kStreamChunk, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        w.hs_pin[i] = nullptr;
        return fail(SHAPE3D_ENOMEM, "pinned host allocation failed");
      }
    }
  }
  return SHAPE3D_OK;
}

bool host_pinned(const void* p) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeHost;
}

// Handshake between the calling thread and the staging thread.
struct StreamSync {
  std::mutex mu;
  std::condition_variable cv;
  long long staged = -1;  // volumes whose copies are enqueued (and event recorded)
  long long used = -1;    // volumes whose "used" event is recorded
  int error = 0;          // a HIP failure of the staging thread
  bool stop = false;      // the calling thread gave up
};

void host_stream_stager(Workspace* w, const void* const* vols, const size_t* bytes, const bool* pinned, int64_t n,
                        StreamSync* S) {
  (void)hipSetDevice(w->device);
  auto ok = [&](hipError_t e) {
    if (e == hipSuccess) return true;
    std::lock_guard<std::mutex> lk(S->mu);
    S->error = (int)e;
    S->cv.notify_all();
    return false;
  };
  bool chunk_used[2] = {false, false};
  int chunk = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int b = (int)(i & 1);
    {
      // volume i reuses the device buffer of volume i - 2: its compute must be enqueued first
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait(lk, [&] { return S->stop || S->used >= i - 2; });
      if (S->stop) return;
    }
    if (i >= 2 && !ok(hipStreamWaitEvent(w->hs_copy, w->hs_ev[2 + b], 0))) return;
    char* dst = (char*)w->hs_vol[b].p;
    if (pinned[i] || bytes[i] == 0) {
      if (bytes[i] && !ok(hipMemcpyAsync(dst, vols[i], bytes[i], hipMemcpyHostToDevice, w->hs_copy))) return;
    } else {
      for (size_t off = 0; off < bytes[i]; off += kStreamChunk) {
        const size_t len = std::min(kStreamChunk, bytes[i] - off);
        if (chunk_used[chunk] && !ok(hipEventSynchronize(w->hs_ev[4 + chunk]))) return;
        memcpy(w->hs_pin[chunk], (const char*)vols[i] + off, len);
        if (!ok(hipMemcpyAsync(dst + off, w->hs_pin[chunk], len, hipMemcpyHostToDevice, w->hs_copy))) return;
        if (!ok(hipEventRecord(w->hs_ev[4 + chunk], w->hs_copy))) return;
        chunk_used[chunk] = true;
        chunk ^= 1;
      }
    }
    if (!ok(hipEventRecord(w->hs_ev[b], w->hs_copy))) return;
    std::lock_guard<std::mutex> lk(S->mu);
    S->staged = i;
    S->cv.notify_all();
  }
}

int host_stream_impl(const void* const* vols, int dtype, const int64_t* dims, const double* spacing, int64_t n,
                     double* out, int* status, int flags, hipStream_t st) {
  if (!vols || !dims || !spacing || !out || !status || n < 1) return fail(SHAPE3D_EINVAL, "null argument or no volume");
  if (dtype != SHAPE3D_U8 && dtype != SHAPE3D_F32) return fail(SHAPE3D_EINVAL, "dtype must be SHAPE3D_U8 or SHAPE3D_F32");
  const bool cls = (flags & SHAPE3D_SHAPE_CLASS) != 0;
  const int nf = cls ? SHAPE3D_N_CLASS : 6;
  std::vector<size_t> bytes((size_t)n, 0);
  std::unique_ptr<bool[]> pinned(new bool[(size_t)n]);
  size_t max_bytes = 0;
  bool any_pageable = false;
  int rc;
  for (int64_t i = 0; i < n; ++i) {
    if (!vols[i]) return fail(SHAPE3D_EINVAL, "null volume " + std::to_string(i));
    if ((rc = check_dims_spacing(dims + 3 * i, spacing + 3 * i))) return rc;
    bytes[i] = (size_t)dims[3 * i] * (size_t)dims[3 * i + 1] * (size_t)dims[3 * i + 2] * (dtype == SHAPE3D_U8 ? 1 : 4);
    pinned[i] = host_pinned(vols[i]);
    any_pageable |= !pinned[i];
    max_bytes = std::max(max_bytes, bytes[i]);
  }
  Workspace* wp = nullptr;
  if ((rc = get_workspace(&wp))) return rc;
  Workspace& w = *wp;
  if ((rc = host_stream_buffers(w, max_bytes, any_pageable))) return rc;
  StreamSync S;
  std::thread stager(host_stream_stager, &w, vols, bytes.data(), pinned.get(), n, &S);
  int result = SHAPE3D_OK;
  for (int64_t i = 0; i < n; ++i) {
    const int b = (int)(i & 1);
    {
      std::unique_lock<std::mutex> lk(S.mu);
      S.cv.wait(lk, [&] { return S.error || S.staged >= i; });
      if (S.error) {
        result = fail(SHAPE3D_EHIP, std::string("HIP error while copying a volume: ") +
                                        hipGetErrorString((hipError_t)S.error));
        break;
      }
    }
    hipError_t e = hipStreamWaitEvent(st, w.hs_ev[b], 0);
    if (e != hipSuccess) {
      result = fail(SHAPE3D_EHIP, hipGetErrorString(e));
      break;
    }
    double* o = out + (size_t)nf * (size_t)i;
    const int r = shape3d_impl(w.hs_vol[b].p, dtype, dims + 3 * i, spacing + 3 * i, o, nullptr, 0, st, nullptr, cls);
    status[i] = r;
    if (r < 0)
      for (int f = 0; f < nf; ++f) o[f] = 0.0;
    if (r == SHAPE3D_EHIP || r == SHAPE3D_ENOMEM) {
      result = r;
      break;
    }
    e = hipEventRecord(w.hs_ev[2 + b], st);
    if (e != hipSuccess) {
      result = fail(SHAPE3D_EHIP, hipGetErrorString(e));
      break;
    }
    std::lock_guard<std::mutex> lk(S.mu);
    S.used = i;
    S.cv.notify_all();
  }
  {
    std::lock_guard<std::mutex> lk(S.mu);
    S.stop = true;
    S.cv.notify_all();
  }
  stager.join();
  // the copy stream may still hold copies of volumes that were not computed
  const hipError_t e = hipStreamSynchronize(w.hs_copy);
  if (result == SHAPE3D_OK && e != hipSuccess) result = fail(SHAPE3D_EHIP, hipGetErrorString(e));
  if (result == SHAPE3D_OK) g_err.clear();
  return result;
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
  return shape3d_batched_ex(base, dtype, rois, n_rois, out, status, nullptr, flags & SHAPE3D_BATCH_GRAPH, stream);
}

int shape3d_batched_ex(const void* base, int dtype, const shape3d_roi* rois, int64_t n_rois, double* out,
                       int* status, shape3d_stats* stats, int flags, void* stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!out || !status) return fail(SHAPE3D_EINVAL, "null output");
  if (flags & ~(SHAPE3D_BATCH_GRAPH | SHAPE3D_SHAPE_CLASS)) return fail(SHAPE3D_EINVAL, "unknown flags");
  const RoiResult* hres = nullptr;
  const int rc = batched_impl(base, dtype, rois, n_rois, flags, (hipStream_t)stream, &hres);
  if (rc < 0 && !hres) return rc;
  const bool cls = (flags & SHAPE3D_SHAPE_CLASS) != 0;
  const int nf = cls ? SHAPE3D_N_CLASS : 6;
  for (int64_t r = 0; r < n_rois; ++r) {
    for (int f = 0; f < 6; ++f) out[nf * r + f] = hres[r].out[f];
    for (int f = 6; f < nf; ++f) out[nf * r + f] = hres[r].shape[f - 6];
    status[r] = hres[r].status;
    if (stats) fill_stats(&stats[r], hres[r], nullptr);
  }
  if (rc < 0) return rc;
  g_err.clear();
  return SHAPE3D_OK;
}

int shape3d_class(const void* vol, int dtype, const int64_t dims[3], const double spacing[3],
                  double out[SHAPE3D_N_CLASS], shape3d_stats* stats, void* stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  return shape3d_impl(vol, dtype, dims, spacing, out, stats, 0, (hipStream_t)stream, nullptr, true);
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
  if ((rc = ensure_layout_bufs(w, Bt, dtype))) return rc;
  long long tcap = 0;
  if ((rc = ensure_staging(w, dtype, staging_guess(Bt), &tcap))) return rc;
  Ptrs P = w.ptrs();
  if ((rc = upload_rois(w, P, Bt, dtype, nullptr, st))) return rc;
  char* h = (char*)w.host;
  long long* th = (long long*)h;
  RoiMeta* mh = (RoiMeta*)(h + 1024);
  for (int pass = 0;; ++pass) {
    if ((rc = launch_head(P, Bt, dtype, tcap, st))) return rc;
    HIPCK(hipMemcpyAsync(th, P.p[W_TOTALS], sizeof(long long) * 9, hipMemcpyDeviceToHost, st));
    HIPCK(hipMemcpyAsync(mh, P.p[W_META], sizeof(RoiMeta), hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    if (th[8] <= tcap || pass > 0) break;
    if ((rc = ensure_staging(w, dtype, th[8], &tcap))) return rc;
    P = w.ptrs();
  }
  if (th[8] > tcap) return fail(SHAPE3D_EINTERNAL, "the mesh pass's staging list overflowed twice");
  const long long V = mh->V;
  *n_out = V;
  if (V > cap) return fail(SHAPE3D_ECAPACITY, "vertex buffer too small");
  if (V == 0) return SHAPE3D_EMPTY;
  Sizes S;
  if ((rc = ensure_vertex_bufs(w, Bt, dtype, th[0], S))) return rc;
  P = w.ptrs();
  if ((rc = launch_rows(P, Bt, dtype, S.rows0, tcap, g_tune.kernel == 1 ? P.as<uint4>(W_POSH) : nullptr, st)))
    return rc;
  HIPCK(launch_export_vertices(P.as<const unsigned long long>(W_KEY),
                               dtype == SHAPE3D_F32 ? P.as<const double>(W_TSOFT) : nullptr,
                               P.as<const RoiMeta>(W_META), P.as<const Roi>(W_ROIS), (long long*)ids, pos, V, st));
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

int shape3d_workspace_size(const int64_t dims[3], int dtype, size_t* bytes) {
  return shape3d_workspace_size_v(dims, dtype, -1, bytes);
}

int shape3d_workspace_size_v(const int64_t dims[3], int dtype, int64_t max_vertices, size_t* bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!dims) return fail(SHAPE3D_EINVAL, "null argument");
  const double one[3] = {1.0, 1.0, 1.0};
  int rc = check_dims_spacing(dims, one);
  if (rc) return rc;
  Batch Bt;
  batch_add(Bt, nullptr, dims, one);
  return workspace_size_impl(Bt, dtype, max_vertices < 0 ? -1 : max_vertices, bytes);
}

int shape3d_batched_workspace_size(int64_t n_rois, const int64_t max_dims[3], int dtype, int64_t max_vertices,
                                   size_t* bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!max_dims || n_rois < 1 || n_rois > SHAPE3D_MAX_ROIS) return fail(SHAPE3D_EINVAL, "bad batch shape");
  Batch Bt;
  int rc = batch_bounds(Bt, n_rois, max_dims);
  if (rc) return rc;
  return workspace_size_impl(Bt, dtype, max_vertices < 0 ? -1 : max_vertices, bytes);
}

int shape3d_ex_async(const void* vol, int dtype, const int64_t dims[3], const double spacing[3], double* out,
                     int* status, void* workspace, size_t ws_bytes, void* stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  int rc = check_args(vol, dtype, dims, spacing);
  if (rc) return rc;
  if ((rc = check_device_span(out, sizeof(double) * 6, "out"))) return rc;
  if ((rc = check_device_span(status, sizeof(int), "status"))) return rc;
  if ((rc = check_device_span(workspace, ws_bytes, "workspace"))) return rc;
  int dev = 0, cu = 0;
  HIPCK(hipGetDevice(&dev));
  if ((rc = device_cu_count(dev, &cu))) return rc;
  Batch Bt;
  batch_add(Bt, vol, dims, spacing);
  rc = run_fixed(Bt, dtype, &Bt.rois[0], nullptr, workspace, ws_bytes, cu, out, status, (hipStream_t)stream);
  if (!rc) g_err.clear();
  return rc;
}

int shape3d_noalloc(const void* vol, int dtype, const int64_t dims[3], const double spacing[3], double* out,
                    int* status, void* stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  int rc = check_args(vol, dtype, dims, spacing);
  if (rc) return rc;
  if ((double)dims[0] * (double)dims[1] * (double)dims[2] > (double)SHAPE3D_NOALLOC_MAX_VOXELS)
    return fail(SHAPE3D_ECAPACITY, "input larger than the no-allocation limit of SHAPE3D_NOALLOC_MAX_VOXELS voxels");
  if ((rc = check_device_span(out, sizeof(double) * 6, "out"))) return rc;
  if ((rc = check_device_span(status, sizeof(int), "status"))) return rc;
  int dev = 0, cu = 0;
  HIPCK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices) return fail(SHAPE3D_ENODEV, "device index beyond the scratch table");
  if (!g_scratch[dev]) {  // once per device, with that device current
    void* ptr = nullptr;
    HIPCK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(SHAPE3D_EHIP, "no device address for the scratch array");
    g_scratch[dev] = ptr;
  }
  if ((rc = device_cu_count(dev, &cu))) return rc;
  // a one-ROI batch built without heap allocation (no ROI vector)
  Batch Bt;
  Roi R;
  memset(&R, 0, sizeof(R));
  const long long d[3] = {dims[0], dims[1], dims[2]};
  const long long nb = roi_fill(R, vol, d, spacing, 0, 0, 0);
  R.brick_begin = 0;
  R.brick_end = nb;
  roi_set_buckets(R, 0);
  Bt.n_rois = 1;
  Bt.nbricks = nb;
  Bt.n_buckets = roi_buckets(R.d);
  Bt.max_G = R.G;
  rc = run_fixed(Bt, dtype, &R, nullptr, g_scratch[dev], (size_t)SHAPE3D_NOALLOC_SCRATCH_BYTES, cu, out, status,
                 (hipStream_t)stream);
  if (!rc) g_err.clear();
  return rc;
}

int shape3d_batched_dev(const void* base, int dtype, const shape3d_roi_ex* rois, int64_t n_rois,
                        const int64_t max_dims[3], double* out, int* status, void* workspace, size_t ws_bytes,
                        int flags, void* stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (flags & ~(SHAPE3D_BATCH_GRAPH | SHAPE3D_SHAPE_CLASS)) return fail(SHAPE3D_EINVAL, "unknown flags");
  return batched_dev_impl(base, dtype, rois, n_rois, max_dims, out, status, workspace, ws_bytes, flags,
                          (hipStream_t)stream);
}

int shape3d_host_stream(const void* const* vols, int dtype, const int64_t* dims, const double* spacing, int64_t n,
                        double* out, int* status, int flags, void* stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (flags & ~SHAPE3D_SHAPE_CLASS) return fail(SHAPE3D_EINVAL, "unknown flags");
  return host_stream_impl(vols, dtype, dims, spacing, n, out, status, flags, (hipStream_t)stream);
}

int shape3d_label_rois(const uint8_t* labels, const int64_t dims[3], const double spacing[3], int32_t max_label,
                       shape3d_roi_ex* rois, int64_t* voxel_counts, int64_t* max_dims, void* stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (max_label < 1 || max_label > 255) return fail(SHAPE3D_EINVAL, "max_label must be in 1..255");
  int rc = check_args(labels, SHAPE3D_U8, dims, spacing);
  if (rc) return rc;
  if ((rc = check_device_span(rois, sizeof(shape3d_roi_ex) * (size_t)max_label, "ROI table"))) return rc;
  if ((uintptr_t)rois % 8) return fail(SHAPE3D_EINVAL, "misaligned ROI table");
  if (voxel_counts && (rc = check_device_span(voxel_counts, sizeof(int64_t) * (size_t)max_label, "voxel_counts")))
    return rc;
  if (max_dims && (rc = check_device_span(max_dims, sizeof(int64_t) * 3, "max_dims"))) return rc;
  int dev = 0, cu = 0;
  HIPCK(hipGetDevice(&dev));
  if ((rc = device_cu_count(dev, &cu))) return rc;
  const long long d[3] = {dims[0], dims[1], dims[2]};
  HIPCK(launch_label_rois(labels, d, spacing, max_label, (RoiDesc*)rois, (long long*)voxel_counts,
                          (long long*)max_dims, cu, (hipStream_t)stream));
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
    drop_graphs(*w);
    if (w->graph_stream) (void)hipStreamDestroy(w->graph_stream);
    for (Buf& b : w->buf)
      if (b.p) (void)hipFree(b.p);
    for (Buf* b : w->soft_bufs())
      if (b->p) (void)hipFree(b->p);
    if (w->host) (void)hipHostFree(w->host);
    if (w->small_slots.p) (void)hipFree(w->small_slots.p);
    for (int i = 0; i < 2; ++i) {
      if (w->hs_vol[i].p) (void)hipFree(w->hs_vol[i].p);
      if (w->hs_pin[i]) (void)hipHostFree(w->hs_pin[i]);
    }
    if (w->hs_copy) {
      (void)hipStreamDestroy(w->hs_copy);
      for (hipEvent_t e : w->hs_ev) (void)hipEventDestroy(e);
    }
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
  t->prune = g_tune.prune;
  t->small_path = g_tune.small_path;
  return SHAPE3D_OK;
}

int shape3d_set_tuning(const shape3d_tuning* t) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!t) return fail(SHAPE3D_EINVAL, "null argument");
  const Tuning c{t->itile_blocks, t->jchunk_blocks, t->blocks_per_cu, t->kernel, t->prune, t->small_path};
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
  best->prune = b.prune;
  best->small_path = b.small_path;
  *best_ms = ms;
  g_err.clear();
  return SHAPE3D_OK;
}

int shape3d_version(void) { return 103; }

}  // extern "C"
