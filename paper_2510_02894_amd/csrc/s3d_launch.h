// s3d_launch.h -- host-side launchers of the kernels (one per pipeline step).
#pragma once
#include <hip/hip_runtime.h>

#include "s3d_internal.h"

namespace s3d {

// Per-ROI result record written by the finalisation kernel.
struct RoiResult {
  double out[6];
  double shape[11];  // the other Shape-class members (when moments were summed), order of SHAPE3D_CLASS_*
  long long n_in;    // inside voxels (when moments were summed)
  double vol_signed;
  long long V, T;
  long long ids[4][2];
  long long rows[4][2];
  long long cand[4];
  long long pairs2d;
  int status;
  int pad_;
};

// The small-mesh path (single ROIs): the four maximum squared distances
// (FP64 bits), the smallest id pair at each (id_lo * 2^32 + id_hi), the
// in-plane pair count and the ticket that finds the pair kernels' last
// workgroup.
struct SmallAcc {
  unsigned long long gmax[4];
  unsigned long long key[4];
  unsigned long long pairs2d;
  unsigned int ticket;
  unsigned int pad_;
};
constexpr long long kSmallMaxV = 16384;         // largest mesh the small path evaluates
constexpr long long kSmallMaxVoxels = 1ll << 22; // larger ROIs go straight to the general path
constexpr int kSmallOverflow = -100;             // status: more vertices than kSmallMaxV

// mesh.hip
// Dynamic LDS of the mesh kernels for ROIs with at most max_G row-groups per row.
size_t mesh_lds_bytes(int max_G);
// The small path's head (ROI record, cleared counts, case areas) and the
// mesh pass alone (no clearing, no case areas).
hipError_t launch_small_head(int dtype, const Roi& R, Roi* rois, long long* totals, SmallAcc* acc,
                             double* case_area, hipStream_t st);
hipError_t launch_mesh_core(int dtype, const Roi* rois, int n_rois, long long nbricks, int max_G,
                            double* case_area, BrickPart* part, unsigned long long* tmpkey, double* tmpt,
                            long long tmp_cap, long long* totals, int moments, hipStream_t st);
// small.hip: every pair of the staged vertices exactly (vmax at most, at
// most kSmallMaxV), in two persistent kernels of n_groups workgroups, then
// the ROI's result in res[0].  acc: small_acc_bytes() of device memory (the
// accumulators, then per-tile maxima).
size_t small_acc_bytes();
hipError_t launch_small_pairs(int dtype, const Roi* rois, const BrickPart* part, long long nbricks,
                              const double* case_area, const unsigned long long* tmpkey, const double* tmpt,
                              const long long* totals, long long vmax, SmallAcc* acc, int n_groups,
                              RoiResult* res, hipStream_t st);

// The mesh pass (one read of the volume): clears counters[0, n_counters),
// then per brick its BrickPart and its vertices' keys (and soft t) in the
// staging list (rows below tmp_cap are written; totals[8] counts all).
// case_area: [n_rois * 512] scratch for the binary masks' per-case areas and
// active-cube counts (case_hist);
// moments: also the inside-voxel moments;
// bmap: [nbricks] scratch for the brick -> ROI map of a batch (unused, and may
// be null, for one ROI).
hipError_t launch_mesh_pass(int dtype, const Roi* rois, int n_rois, long long nbricks, int max_G,
                            double* case_area, BrickPart* part, unsigned int* counters, int n_counters,
                            unsigned long long* tmpkey, double* tmpt, long long tmp_cap, long long* totals,
                            int moments, int* bmap, hipStream_t st);
// Per-ROI totals and each brick's first row within its ROI (brick_voff);
// prune_min_v: ROIs with at least this many vertices get the pruning pass's column-pair offsets.
hipError_t launch_mesh_totals(const Roi* rois, int n_rois, long long nbricks, int dtype, const double* case_area,
                              const BrickPart* part, long long* brick_voff, RoiMeta* meta, long long* totals,
                              int moments, int prune_min_v, hipStream_t st);
// The capacity check (rows0_cap rows; *overflow raised and every ROI emptied
// beyond it), the 3D segments, and layout 0 from the staging list (tmp_cap
// rows): keys, soft t, pair-pass operands (pos, or posh when set), orig and
// block tags.
hipError_t launch_mesh_rows(const Roi* rois, int n_rois, long long nbricks, const BrickPart* part,
                            const long long* brick_voff, RoiMeta* meta, long long* totals, long long rows0_cap,
                            const unsigned long long* tmpkey, const double* tmpt, long long tmp_cap,
                            unsigned long long* key, double* tsoft, float* pos, uint4* posh, int* orig, int* blkseg,
                            Seg* segs, unsigned int* overflow, const int* bmap, hipStream_t st);

// labels.hip: the ROI table of labels 1..max_label of a dense uint8 label map
// (crop to each label's box, select the label), the voxel counts (counts,
// may be null) and the largest crop (max_dims, may be null).  The table's
// entries also hold the boxes while they are built.
hipError_t launch_label_rois(const unsigned char* lab, const long long dims[3], const double spacing[3],
                             int max_label, RoiDesc* rois, long long* counts, long long* max_dims, int cu_count,
                             hipStream_t st);

// ROI tables on the device: a caller's descriptors planned and validated in
// one workgroup (plan[0] = bricks, plan[1] = buckets), or one ROI by value.
hipError_t launch_plan_rois(const RoiDesc* in, int n, int dtype, const long long max_dims[3], const void* base,
                            long long alloc_elems, Roi* out, long long* plan, hipStream_t st);
hipError_t launch_set_roi(const Roi& R, Roi* out, hipStream_t st);

// scan.hip: exclusive scan of n int64 (n known on the host); total -> *total.
// With n_dev set, only the first min(n, *n_dev) elements are scanned (a count
// known on the device only): later tiles cost an early exit and their outputs
// are left unwritten.  tmp must hold scan_tmp_elems(n) int64.
long long scan_tmp_elems(long long n);
hipError_t launch_scan(const long long* in, long long* out, long long n, long long* total, long long* tmp,
                       hipStream_t st, const unsigned int* n_dev = nullptr);
hipError_t launch_fill_u32(unsigned int* p, unsigned int v, long long n, hipStream_t st);
hipError_t launch_fill_i64(long long* p, long long v, long long n, hipStream_t st);

// Tile sizes of the pair pass (chosen by the autotuner; results do not depend on them).
struct Tuning {
  int itile;          // 16-row blocks per wave: 2, 4 or 8 (kernel 1: 4 or 8)
  int jchunk;         // 16-row column blocks per work item: 64, 128, 256 or 512
  int blocks_per_cu;  // persistent workgroups per CU (0: as many as fit)
  int kernel;         // 0: FP32 16x16x4 MFMA; 1: split-f16 32x32x16 MFMA
  int prune;          // 1: skip 3D pair tiles that cannot reach the diameter (kernel 1); 0: all pairs
  int small_path;     // 1: small single ROIs take the exact all-pairs kernel after the mesh pass
};

// Buffers of the diameter passes.
// What a per-brick kernel needs to find a brick's vertices in layout 0.
struct BrickArgs {
  const Roi* rois;
  int n_rois;
  const RoiMeta* meta;
  const BrickPart* part;       // [nbricks] the mesh pass's per-brick records
  const long long* brick_voff;  // [nbricks] each brick's first vertex within its ROI
  const int* bmap;             // [nbricks] brick -> ROI map, or null (then the ROI table is searched)
  long long nbricks;
};

struct PairBufs {
  const Roi* rois;
  int n_rois;
  long long nbricks;            // bricks of the mesh pass (its grid)
  const BrickPart* part;        // [nbricks]
  const long long* brick_voff;  // [nbricks]
  const int* bmap;              // [nbricks] or null
  int brick_win;                // LDS plane-key windows of the per-brick bucket kernels (at most 2,048)
  const RoiMeta* meta;
  const unsigned long long* key;
  const double* tsoft;  // null for binary masks
  float* pos;
  uint4* posh;          // split-f16 B operands, 32 B per row (kernel 1)
  int* orig;
  float* rowmax;
  int* blkseg;
  Seg* segs;
  long long rows0;      // layout-0 rows (host copy)
  long long n_buckets;  // plane buckets of all ROIs
  unsigned int* bcnt;   // [n_buckets]
  unsigned int* bcur;   // [n_buckets]
  long long* bsz;       // [n_buckets]
  long long* bflag;     // [n_buckets]
  long long* brow;      // [n_buckets]
  long long* bseg;      // [n_buckets]
  int4* bbox;           // [n_buckets] key-coordinate boxes of the plane buckets (pruning)
  int* bgroup;          // [n_buckets] group roi * 4 + 1 + axis of each plane bucket
  long long seg_cap;    // n_rois + n_buckets
  long long* ncol;      // [seg_cap]
  long long* colbase;   // [seg_cap]
  long long col_cap;
  Col* cols;            // [col_cap]
  long long* nitem;     // [col_cap]
  long long* itembase;  // [col_cap]
  long long* totals;    // device scalars: see pairs.hip
  long long* scan_tmp;
  unsigned int* counters;  // [1] candidates, [2] overflow flag; pair-pass work counters from word kWorkStride
  GroupRes* gres;          // [4 * n_rois]
  long long cand_cap;      // candidate capacity: every row could be one
  int* cand;               // [cand_cap]
  long long* cand_nch;     // [cand_cap] chunks of each candidate's segment
  long long* cand_chbase;  // [cand_cap] prefix sum of cand_nch
  long long max_rows_seg;  // bound on rows of one segment
  long long rows_bound;    // bound on rows of all layouts (allocation)
  Tuning tune;
  RoiResult* res;          // [n_rois]
  long long* pairs2d;      // [n_rois] in-plane pairs n*(n-1)/2 summed over buckets
  int cu_count;
  bool moments;            // RoiMeta holds inside-voxel moments: finalise the whole Shape class
  bool ids32;              // every canonical vertex id of the call is below 2^32 (packed tie-break)
  // 3D pruning (prune.hip), kernel 1 only: when `prune` is set the 3D
  // segments run from the pruned item list instead of the work list
  bool prune;
  int prune_min_v;         // ROIs with at least this many vertices are pruned, the others run all pairs
  BlkRec* blkrec;          // [rows0 / 32] per 32-row block of layout 0
  RoiSeed* rseed;          // [n_rois]
  PItem* pitems;           // [pitem_cap]
  long long pitem_cap;
};

// soft.hip: adjoint of the soft-mask forward pass, for a table of ROIs.
// Cubes u in [-1, d-1]^3 have the flat index cube(u) = ((u0 + 1) (d1 + 1) +
// u1 + 1) (d2 + 1) + u2 + 1; grid edge (u, u + e_a) has the edge-field slot
// field_begin + 3 cube(u) + a.  Local indices are below 2^31 (checked on the
// host), so the kernels divide with 32-bit magic numbers: floor(n / D) =
// (n * m) >> sh with sh = 31 + ceil(log2 D) and m = floor(2^sh / D) + 1.
constexpr int kCubeBlock = 4096;   // cubes per workgroup of the edge pass (16 per thread)
constexpr int kVoxPer = 4;         // voxels per thread of the gather pass (256 apart)
constexpr int kVoxBlock = 256 * kVoxPer;  // voxels per workgroup of the gather pass

struct SoftBwdRoi {
  const float* p;             // the ROI's probabilities (d0, d1, d2)
  float* grad;                // dL/dp, same layout
  int d[3];
  int pad_;
  double s[3];
  double o[3];                // origin of the signed volume sum (array centre)
  double g_area;              // dL/dSurfaceArea
  double g_vol_signed;        // dL/dMeshVolume * sign(signed volume)
  double gdiam[4];            // dL/dD_f / D_f (0 if the feature has no pair)
  long long pair_ids[4][2];   // canonical ids of the maximising pairs, -1 if none
  long long field_begin;      // first slot of the ROI in the edge field
  long long cblk_begin;       // first workgroup of the edge pass
  long long vblk_begin;       // first workgroup of the gather pass
  unsigned int n_cubes;       // (d0 + 1)(d1 + 1)(d2 + 1)
  unsigned int n_vox;         // d0 d1 d2
  unsigned int m_cplane, m_c2, m_plane, m_d2;  // magic numbers for (d1+1)(d2+1), d2+1, d1 d2, d2
  int sh_cplane, sh_c2, sh_plane, sh_d2;
};

struct SoftBwdBufs {
  const SoftBwdRoi* rois;     // [n_rois], DEVICE
  int n_rois;
  long long n_cblocks;        // workgroups of the edge pass
  long long n_vblocks;        // workgroups of the gather pass
  long long cap;              // crossing-edge capacity (the forward pass's vertex count)
  unsigned long long* edges;  // [cap] crossing edges: ROI index << 40 | local field slot
  float* field;               // edge field: (dL/dx_v)_a * s_a at crossing edges (other slots unused)
  long long n_field;          // slots of the edge field
  long long* counters;        // [0] edges reserved
  int cu_count;
  int* blk_roi;               // [n_cblocks + n_vblocks] ROI of each edge-pass then gather-pass
                              // workgroup, or null (then found by binary search)
};
hipError_t launch_soft_backward(const SoftBwdBufs& B, hipStream_t st);

// pairs.hip
uint4* split_rows(const PairBufs& B);  // split-f16 operand rows (kernel 1), else null
hipError_t launch_buckets(const PairBufs& B, hipStream_t st);       // plane buckets, segments, work list
// prune.hip: boxes, lower bound and the pruned 3D work items (B.prune set)
hipError_t launch_prune(const PairBufs& B, hipStream_t st);
hipError_t launch_pair_maxima(const PairBufs& B, hipStream_t st);   // MFMA pass over the work list
hipError_t launch_init_groups(const PairBufs& B, hipStream_t st);   // reset group results, pair-pass counters, row maxima
hipError_t launch_refine(const PairBufs& B, hipStream_t st);        // candidates + exact FP64 passes
hipError_t launch_finalize(const PairBufs& B, hipStream_t st);      // per-ROI results
// res -> out[nf * n_rois] (nf = 6, or 17 for the whole Shape class; not written for a negative
// status) and status[n_rois] (may be null), on the device
hipError_t launch_results_out(const RoiResult* res, int n_rois, double* out, int* status, int nf, hipStream_t st);
hipError_t launch_export_vertices(const unsigned long long* key, const double* tsoft, const RoiMeta* meta,
                                  const Roi* rois, long long* ids, double* pos, long long V, hipStream_t st);

}  // namespace s3d
