/*
 * shape3d.h -- C ABI of the MI355X (gfx950) 3D shape-feature library.
 *
 * The library computes the six mesh-based shape features of a region of
 * interest (ROI) that the paper accelerates (Sec. 2, "PyRadiomics-cuda
 * design"): the mesh volume and surface area of a marching-cubes surface
 * ("Marching cubes fused parallel kernels" paragraph), and the maximum
 * distance between mesh vertices in 3D and within each axis-aligned plane
 * ("Parallel diameter calculation" paragraph; the planar diameters of the
 * feature list in Sec. 2).
 *
 * Conventions shared by every entry point:
 *   - the volume is C-contiguous with shape (d0, d1, d2) (axis 0 slowest);
 *     dims and spacing are given in that same axis order; spacing in mm;
 *   - dtype SHAPE3D_U8: uint8 mask, voxel inside iff value != 0, mesh
 *     vertices at edge midpoints; dtype SHAPE3D_F32: float32 probabilities,
 *     inside iff p > 0.5, vertices linearly interpolated at the 0.5 level;
 *   - voxels outside the array count as outside (one-voxel zero pad);
 *   - features, in order: MeshVolume (mm^3, absolute value of the signed
 *     tetrahedron sum), SurfaceArea (mm^2), Maximum3DDiameter,
 *     Maximum2DDiameterSlice (vertex pairs on a common plane of axis 0),
 *     ...Column (axis 1), ...Row (axis 2), all in mm;
 *   - a mesh vertex is identified by its canonical id
 *     3 * (((u0+1)*(d1+2) + (u1+1))*(d2+2) + (u2+1)) + a for the grid edge
 *     (u, u + e_a) it lies on;
 *   - the maximising pair of a diameter is the pair with the largest
 *     distance and, among equal distances, the lexicographically smallest
 *     pair of canonical ids.
 *
 * Pointers documented as DEVICE point to memory on the current HIP device;
 * HOST pointers to ordinary host memory.  `stream` is a hipStream_t (NULL =
 * the null stream).  The caller owns every buffer it passes.  The library
 * owns a workspace per device that grows on demand and is kept between calls
 * (shape3d_release frees it).  Calls are serialised by an internal lock;
 * device buffers given to a call must stay valid until it returns.
 *
 * Every function returns a status.  On a failure (negative status) the
 * outputs are left untouched and shape3d_last_error() describes the cause.
 * There is no CPU fallback: without a usable GPU the functions return
 * SHAPE3D_ENODEV.
 */
#ifndef SHAPE3D_H
#define SHAPE3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SHAPE3D_OK 0
#define SHAPE3D_EMPTY 1      /* no foreground voxel: features are all 0 */
#define SHAPE3D_EINVAL (-1)  /* bad argument (null pointer, dims, spacing, dtype) */
#define SHAPE3D_ENODEV (-2)  /* no usable HIP device */
#define SHAPE3D_EHIP (-3)    /* a HIP runtime call failed */
#define SHAPE3D_ECAPACITY (-4) /* an internal bound was exceeded */
#define SHAPE3D_ENOMEM (-5)  /* device allocation failed */
#define SHAPE3D_EINTERNAL (-6) /* an internal consistency check failed */

#define SHAPE3D_U8 0
#define SHAPE3D_F32 1

/* Largest accepted extent of axes 0 and 1, and of axis 2 (the contiguous axis,
   whose rows one workgroup of the mesh pass stages in LDS). */
#define SHAPE3D_MAX_DIM 1000000
#define SHAPE3D_MAX_DIM2 32767

/* Per-call statistics (optional output of shape3d_ex). */
typedef struct {
  int64_t n_vertices;      /* V: mesh vertices (crossing grid edges) */
  int64_t n_triangles;     /* T: mesh triangles */
  int64_t pair_ids[4][2];  /* canonical ids of the maximising pair: 3D, slice, column, row (-1: none) */
  int64_t pairs_3d;        /* V*(V-1)/2 */
  int64_t pairs_2d;        /* sum over planes of n*(n-1)/2 */
  int64_t candidates[4];   /* rows re-examined in FP64 per diameter */
  float ms[8];             /* device time per phase (ms), filled when timing != 0:
                              0 mesh pass (one read of the volume) and per-ROI totals,
                              1 vertex rows and pair-pass operands, 2 pruning and plane bucketing,
                              3 pair maxima (MFMA),
                              4 exact refinement, 5 finalisation, 6 whole call, 7 reserved */
} shape3d_stats;

/*
 * shape3d -- the six features of one binary ROI, synchronously.
 *   mask:    DEVICE, uint8 (d0, d1, d2), C-contiguous; nonzero = inside.
 *   dims:    HOST int64[3]; dims[0], dims[1] in [1, SHAPE3D_MAX_DIM],
 *            dims[2] in [1, SHAPE3D_MAX_DIM2].
 *   spacing: HOST double[3]; each finite and > 0.
 *   out:     HOST double[6], the features in the order above.
 * Uses the null stream.  Returns SHAPE3D_OK, SHAPE3D_EMPTY (out all zero) or
 * a negative error.
 */
int shape3d(const uint8_t* mask, const int64_t dims[3], const double spacing[3], double out[6]);

/*
 * shape3d_ex -- as shape3d, for either dtype, on `stream`, with optional
 * statistics.  vol: DEVICE volume of `dtype`.  out: HOST double[6].
 * stats: HOST, may be NULL.  timing: nonzero records per-phase HIP events
 * into stats->ms (costs a few microseconds).  Returns when the results are
 * on the host.
 */
int shape3d_ex(const void* vol, int dtype, const int64_t dims[3], const double spacing[3],
               double out[6], shape3d_stats* stats, int timing, void* stream);

/*
 * shape3d_batched -- the six features of many ROIs in one pass of the
 * pipeline (all ROIs' bricks, vertices, plane buckets and pair tiles share
 * each launch).  The paper computes one ROI per call (Sec. 3 measures cases
 * one by one); a batch lets small ROIs fill the GPU together.
 *   base:   DEVICE pointer; ROI r's volume (dtype, C-contiguous) starts at
 *           base + rois[r].offset elements.  Every ROI must lie inside the
 *           allocation that holds base.
 *   rois:   HOST array of n_rois descriptors (dims and spacing as in shape3d).
 *   n_rois: 1 .. SHAPE3D_MAX_ROIS.
 *   out:    HOST double[6 * n_rois]; status: HOST int[n_rois] (SHAPE3D_OK or
 *           SHAPE3D_EMPTY per ROI).
 *   flags:  SHAPE3D_BATCH_GRAPH records the launch sequence as a hipGraph on
 *           the first call and replays it on later calls with the same base,
 *           dtype and ROI table (the device buffers are sized by the first
 *           call; if a replay finds more vertices than they hold, the call is
 *           re-run eagerly and recorded again).
 * Synchronous on `stream`.  Returns SHAPE3D_OK or a negative error.
 */
typedef struct {
  int64_t offset;     /* element offset of the ROI's volume from base */
  int64_t dims[3];
  double spacing[3];
} shape3d_roi;

#define SHAPE3D_BATCH_GRAPH 1
#define SHAPE3D_MAX_ROIS (1 << 20)

int shape3d_batched(const void* base, int dtype, const shape3d_roi* rois, int64_t n_rois, double* out,
                    int* status, int flags, void* stream);

/*
 * The whole Shape class.  The paper's feature list (Sec. 2) is the six
 * features above; PyRadiomics' Shape class, which the paper accelerates,
 * also has members that are closed forms of MeshVolume V, SurfaceArea A and
 * the number n of inside voxels, and members from the principal axes of the
 * inside voxels.  With the covariance C of the inside voxels' physical
 * coordinates (index * spacing; population covariance, divisor n) and its
 * eigenvalues l_least <= l_minor <= l_major (negative rounding clamped to 0),
 * the SHAPE3D_N_CLASS outputs are, in order:
 *   0-5  the six features above;
 *   6    VoxelVolume            = n s0 s1 s2
 *   7    SurfaceVolumeRatio     = A / V
 *   8    Sphericity             = (36 pi V^2)^(1/3) / A
 *   9    Compactness1           = V / (sqrt(pi) A^(3/2))
 *   10   Compactness2           = 36 pi V^2 / A^3
 *   11   SphericalDisproportion = A / (36 pi V^2)^(1/3)
 *   12   MajorAxisLength        = 4 sqrt(l_major)
 *   13   MinorAxisLength        = 4 sqrt(l_minor)
 *   14   LeastAxisLength        = 4 sqrt(l_least)
 *   15   Elongation             = sqrt(l_minor / l_major)  (0 if l_major = 0)
 *   16   Flatness               = sqrt(l_least / l_major)  (0 if l_major = 0)
 * all 0 for an empty ROI.  The moments are summed exactly in integers in the
 * mesh pass (the same read of the volume), the eigenvalues come from Jacobi
 * rotations in FP64.
 *
 * shape3d_class -- the SHAPE3D_N_CLASS members for one ROI (arguments as
 *   shape3d_ex; out: HOST double[SHAPE3D_N_CLASS]; stats: HOST or NULL).
 *   Synchronous on `stream`.
 *
 * shape3d_batched_ex -- shape3d_batched with per-ROI statistics and flags.
 *   stats: HOST shape3d_stats[n_rois] or NULL: V, T, maximising pairs,
 *          in-plane pair counts and candidate rows of every ROI (ms fields 0).
 *   flags: SHAPE3D_BATCH_GRAPH as shape3d_batched, plus SHAPE3D_SHAPE_CLASS:
 *          out is then HOST double[SHAPE3D_N_CLASS * n_rois] (ROI r's members
 *          at out[SHAPE3D_N_CLASS r ...]); without it double[6 * n_rois].
 *   Other arguments and errors as shape3d_batched.
 */
#define SHAPE3D_SHAPE_CLASS 2
#define SHAPE3D_N_CLASS 17

int shape3d_class(const void* vol, int dtype, const int64_t dims[3], const double spacing[3],
                  double out[SHAPE3D_N_CLASS], shape3d_stats* stats, void* stream);
int shape3d_batched_ex(const void* base, int dtype, const shape3d_roi* rois, int64_t n_rois, double* out,
                       int* status, shape3d_stats* stats, int flags, void* stream);

/*
 * shape3d_vertices -- the mesh vertex set, for verification.
 *   ids:  DEVICE int64[cap]; receives the canonical ids of all V vertices
 *         (in the library's emission order, which is deterministic).
 *   pos:  DEVICE double[3*cap] or NULL; receives their positions (mm,
 *         index * spacing, not centred).
 *   n_out: HOST; receives V.  If V > cap nothing is written to ids/pos and
 *         SHAPE3D_ECAPACITY is returned with *n_out = V.
 */
int shape3d_vertices(const void* vol, int dtype, const int64_t dims[3], const double spacing[3],
                     int64_t* ids, double* pos, int64_t cap, int64_t* n_out, void* stream);

/*
 * Differentiable soft-mask mode.  The paper's mesh pass (Sec. 2, marching
 * cubes on the segmentation threshold) applied to a float32 probability map
 * p with isolevel 0.5: vertices at t = (0.5 - p_u) / (p_b - p_u) along each
 * crossing edge, so the six features are piecewise-smooth functions of p.
 *
 * shape3d_soft_forward -- the features of a soft mask (as shape3d_ex with
 * SHAPE3D_F32) and, in `saved` (HOST, caller-owned), what the backward pass
 * needs: dims, spacing, features, the signed volume, the maximising pairs and
 * the vertex count.
 *   p: DEVICE float32 (d0, d1, d2).  out: HOST double[6].  Synchronous.
 *
 * shape3d_soft_backward -- dL/dp for L = sum_f grad_out[f] * F_f, the exact
 * derivative of the forward pass where the triangulation and the maximising
 * pairs do not change (area and volume through every vertex position, each
 * diameter through its maximising pair; MeshVolume = |signed volume| uses
 * its sign).
 *   p:        DEVICE float32, the same values the forward pass saw.
 *   saved:    HOST, from shape3d_soft_forward on p.
 *   grad_out: HOST double[6], finite.
 *   grad_p:   DEVICE float32 (d0, d1, d2), fully written (0 away from the surface).
 * Synchronous on `stream`.  If p does not have the crossing edges the forward
 * pass counted, SHAPE3D_EINVAL is returned and grad_p is unspecified.
 */
typedef struct {
  int64_t dims[3];
  double spacing[3];
  double features[6];
  double signed_volume;
  int64_t pair_ids[4][2];
  int64_t n_vertices;     /* V of the forward pass: crossing edges of p */
  int status;
} shape3d_soft_saved;

int shape3d_soft_forward(const float* p, const int64_t dims[3], const double spacing[3], double out[6],
                         shape3d_soft_saved* saved, void* stream);
int shape3d_soft_backward(const float* p, const shape3d_soft_saved* saved, const double grad_out[6],
                          float* grad_p, void* stream);

/*
 * Batched soft mode: the two passes above for a table of float32 ROIs, each
 * pass one pipeline over all ROIs (the forward is shape3d_batched's).
 *
 * shape3d_batched_soft_forward
 *   base, rois, n_rois, flags: as shape3d_batched (dtype SHAPE3D_F32).
 *   out:   HOST double[6 * n_rois].
 *   saved: HOST shape3d_soft_saved[n_rois]; saved[r].status is SHAPE3D_OK or
 *          SHAPE3D_EMPTY.
 *
 * shape3d_batched_soft_backward -- dL/dp of every ROI for
 * L = sum_r sum_f grad_out[6 r + f] * F_f(ROI r), in three launches over all
 * ROIs (crossing-edge lists, per-vertex gradients, per-voxel sums).
 *   base, rois, n_rois: as the forward call.
 *   saved:     HOST, from shape3d_batched_soft_forward on the same inputs.
 *   grad_out:  HOST double[6 * n_rois], finite.
 *   grad_base: DEVICE float32; ROI r's gradient is written at
 *              grad_base + rois[r].offset in the ROI's layout (elements
 *              outside every ROI are not touched; ROIs must not overlap).
 * Synchronous on `stream`.  Errors as shape3d_soft_backward.
 */
int shape3d_batched_soft_forward(const float* base, const shape3d_roi* rois, int64_t n_rois, double* out,
                                 shape3d_soft_saved* saved, int flags, void* stream);
int shape3d_batched_soft_backward(const float* base, const shape3d_roi* rois, int64_t n_rois,
                                  const shape3d_soft_saved* saved, const double* grad_out, float* grad_base,
                                  void* stream);

/*
 * Tile sizes of the all-pairs pass and their autotuner.  The paper sizes its
 * diameter kernel by hand for one GPU (Sec. 3, micro-benchmarks of the kernel
 * variants); here the tiles are chosen per workload class by timing.  Tiles
 * change only the order of the work: every result is identical for every
 * valid setting.
 *   itile_blocks:  16-row blocks each wave keeps in registers: 2, 4 or 8
 *                  (kernel 1: 4 or 8).
 *   jchunk_blocks: 16-row column blocks per work item: 64, 128, 256, 512 or
 *                  1024.
 *   blocks_per_cu: persistent workgroups per compute unit, 0 = as many as fit
 *                  (at most 64).
 *   kernel:        0 = FP32 Gram values on the 16x16x4 FP32 matrix cores;
 *                  1 = FP32-accurate Gram values from coordinates split into
 *                  two f16 parts on the 32x32x16 f16 matrix cores.  Both are
 *                  followed by the same exact FP64 refinement.
 *   prune:         (kernel 1) skip the 3D pair tiles whose largest possible
 *                  distance, from the bounding boxes of their vertex blocks,
 *                  stays below a vertex-pair distance found by two
 *                  farthest-point sweeps, and the plane buckets whose box
 *                  diagonal stays below the largest in-plane extent of any
 *                  bucket of their family: 1 = in calls whose largest ROI may
 *                  have 16,384 vertices or more (then the 3D pairs of every
 *                  ROI with 1,024 or more), 2 = always (every ROI), 0 = never
 *                  (all pairs).  Exact: the maximising pairs are never
 *                  skipped, and the FP64 refinement rescans its candidate rows
 *                  against all vertices of their segment, so the results equal
 *                  those of prune = 0.
 * The setting is process-wide (all devices); the default is {8, 1024, 0, 1, 1}
 * (the autotuner's choice on one very large ROI; batches of small ROIs gain
 * about 1 % from jchunk 512).
 *
 * shape3d_get_tuning / shape3d_set_tuning -- read or replace the setting
 * (HOST struct).  Setting drops the graphs recorded by shape3d_batched.
 * Neither needs a device.  SHAPE3D_EINVAL for unsupported values.
 *
 * shape3d_autotune -- runs the batch (as shape3d_batched, eagerly) once per
 * candidate setting (kernel 0 with itile 2, 4, 8 and kernel 1 with itile 4, 8,
 * each with the four jchunk values; `reps` timed runs each, 1..100), keeps
 * the tiling with the shortest pair-pass time (HIP events) and makes it the
 * current setting.  Returns SHAPE3D_EINTERNAL if a candidate changes any
 * result.
 *   cache_path: HOST path of a text file or NULL.  Lines are
 *               "<class> <kernel> <itile> <jchunk> <blocks_per_cu> <ms>", the class
 *               being the dtype and the rounded log2 of the ROI count, of
 *               the total and of the largest vertex count.  A line for the
 *               batch's class is used without timing; otherwise the choice is
 *               appended.
 *   best:       HOST; receives the chosen tiles.  best_ms: HOST; its pair-pass
 *               time (from the cache on a hit).
 * Synchronous on `stream`.
 */
typedef struct {
  int32_t itile_blocks;
  int32_t jchunk_blocks;
  int32_t blocks_per_cu;
  int32_t kernel;
  int32_t prune;  /* kernel 1: 1 (default) prune the 3D pair tiles of large ROIs, 2 always, 0 never */
  int32_t small_path; /* 1 (default): single-ROI calls of at most 2^22 voxels and 16,384 vertices
                         (six features, no phase timing) evaluate all pairs exactly in one kernel
                         after the mesh pass; 0: always the general pipeline.  Results are identical. */
} shape3d_tuning;

int shape3d_get_tuning(shape3d_tuning* t);
int shape3d_set_tuning(const shape3d_tuning* t);
int shape3d_autotune(const void* base, int dtype, const shape3d_roi* rois, int64_t n_rois, int reps,
                     const char* cache_path, shape3d_tuning* best, double* best_ms, void* stream);

/*
 * Caller-provided workspaces and results that stay on the device.
 *
 * The calls above size the library's own device workspace, which means a
 * device-to-host read of the vertex count after the mesh count pass.  The
 * calls below run on a workspace the caller provides (or, for
 * shape3d_batched_dev, optionally on the library's), write their results to
 * device memory and return as soon as the work is enqueued: nothing is read
 * back to the host.  The vertex capacity follows from ws_bytes; a mesh that
 * needs more rows than fit ends with status SHAPE3D_ECAPACITY (out left
 * untouched), never with an out-of-bounds write.  A workspace must not be used
 * by two calls that are in flight at once (calls on one stream are ordered);
 * its contents between calls are unspecified.
 *
 * shape3d_workspace_size -- bytes of a workspace that holds the mesh of any
 *   mask of these dims (every grid edge crossing: an upper bound, about
 *   3 (d0+1)(d1+1)(d2+1) vertex rows of ~110 B).  SHAPE3D_ECAPACITY if such a
 *   mesh exceeds the kernels' 32-bit row indices.
 * shape3d_workspace_size_v -- the same for meshes of at most max_vertices
 *   vertices (max_vertices < 0: the worst case above).  Depends on the current
 *   tuning (the operand layout of the pair pass).
 * shape3d_batched_workspace_size -- the same for a batch of n_rois ROIs, each
 *   at most max_dims, with at most max_vertices vertices in total.
 * None of the three needs a device.
 *
 * shape3d_ex_async -- the six features of one ROI, as shape3d_ex, fully
 * asynchronous on `stream`.
 *   vol, dtype, dims, spacing: as shape3d_ex.
 *   out:       DEVICE double[6], written unless the status is negative.
 *   status:    DEVICE int[1]: SHAPE3D_OK, SHAPE3D_EMPTY or SHAPE3D_ECAPACITY.
 *   workspace: DEVICE, 256-byte aligned, ws_bytes long (shape3d_workspace_size).
 * The return value covers argument errors only (SHAPE3D_ECAPACITY if not even
 * an empty mesh's buffers fit).
 */
int shape3d_workspace_size(const int64_t dims[3], int dtype, size_t* bytes);
int shape3d_workspace_size_v(const int64_t dims[3], int dtype, int64_t max_vertices, size_t* bytes);
int shape3d_batched_workspace_size(int64_t n_rois, const int64_t max_dims[3], int dtype, int64_t max_vertices,
                                   size_t* bytes);
int shape3d_ex_async(const void* vol, int dtype, const int64_t dims[3], const double spacing[3], double* out,
                     int* status, void* workspace, size_t ws_bytes, void* stream);

/*
 * shape3d_batched_dev -- shape3d_batched with the ROI table, the features and
 * the statuses in device memory, so that a batch can be described by earlier
 * device work (for instance a crop to each label's bounding box) and a
 * recorded graph can be replayed on new table contents without any host
 * involvement.
 *   base:     DEVICE; ROI r's voxel (z, y, x) is
 *             base[rois[r].offset + z strides[0] + y strides[1] + x].
 *   rois:     DEVICE shape3d_roi_ex[n_rois].  strides of 0 mean the dense
 *             layout (dims[1] dims[2], dims[2]); otherwise strides[1] >=
 *             dims[2] and strides[0] >= (dims[1] - 1) strides[1] + dims[2].
 *             label (uint8 only): 0 = nonzero voxels are inside; 1..255 =
 *             voxels equal to label are inside (label maps).
 *   max_dims: HOST int64[3], bounds on every ROI's dims (they size the
 *             launches and buffers).  An entry that is out of bounds, reaches
 *             past the allocation holding base, or is otherwise invalid gets
 *             status SHAPE3D_EINVAL; the other ROIs are unaffected.
 *   out:      DEVICE double[6 n_rois], or double[SHAPE3D_N_CLASS n_rois] with
 *             SHAPE3D_SHAPE_CLASS in flags; status: DEVICE int[n_rois].
 *   workspace: DEVICE or NULL.  With a workspace: as shape3d_ex_async (no
 *             host synchronisation; shape3d_batched_workspace_size).  With
 *             NULL the library's workspace is used: the call reads the vertex
 *             row count back once to size it, and with SHAPE3D_BATCH_GRAPH it
 *             records the pipeline (table planning included) the first time
 *             and later replays it for the same base, dtype, table pointer,
 *             n_rois, max_dims and output pointers; a replay whose meshes
 *             exceed the recorded capacity sets every status to
 *             SHAPE3D_ECAPACITY (call without the flag once to resize).
 *             SHAPE3D_SHAPE_CLASS: the whole Shape class per ROI (see
 *             shape3d_class).
 * Enqueued on `stream`; returns without waiting for the results.
 */
typedef struct {
  int64_t offset;      /* element offset of the ROI's voxel (0, 0, 0) from base */
  int64_t dims[3];
  double spacing[3];
  int64_t strides[2];  /* elements between voxels along axes 0 and 1; 0 = dense */
  int32_t label;       /* uint8: 0 = nonzero is inside, else voxels equal to label */
  int32_t reserved;    /* must be 0 */
} shape3d_roi_ex;

int shape3d_batched_dev(const void* base, int dtype, const shape3d_roi_ex* rois, int64_t n_rois,
                        const int64_t max_dims[3], double* out, int* status, void* workspace, size_t ws_bytes,
                        int flags, void* stream);

/*
 * shape3d_host_stream -- the features of n volumes that start in HOST memory,
 * with the host-to-device transfer of volume i + 1 overlapped with the
 * computation of volume i.  The paper copies each input to the device before
 * its kernels run and reports that transfer as a large share of its GPU time
 * (Sec. 3, discussion of the results; Table 2, transfer column): here a
 * staging thread of the library copies on a stream of its own while the
 * calling thread runs the pipeline on `stream`, and two device volumes
 * alternate.  Page-locked sources (hipHostMalloc) are copied by DMA
 * directly; pageable ones pass through two pinned 32 MiB chunks of the
 * library that alternate.
 *   vols:    HOST array of n HOST pointers, each a C-contiguous volume of
 *            dtype (as shape3d_ex) and dims[3 i .. 3 i + 2].
 *   dims, spacing: HOST int64[3 n], double[3 n].
 *   out:     HOST double[6 n], or double[SHAPE3D_N_CLASS n] with
 *            SHAPE3D_SHAPE_CLASS in flags (the only flag).
 *   status:  HOST int[n]: each volume's status (as shape3d_ex; out rows of a
 *            failed volume are 0).
 * Synchronous: returns when every result is in out.  The library keeps two
 * device volumes of the largest size seen (and the pinned chunks) until
 * shape3d_release.  Returns SHAPE3D_EINVAL for bad arguments (checked for
 * every volume before any copy), SHAPE3D_ENOMEM, or SHAPE3D_EHIP if a copy
 * failed.
 */
int shape3d_host_stream(const void* const* vols, int dtype, const int64_t* dims, const double* spacing, int64_t n,
                        double* out, int* status, int flags, void* stream);

/*
 * shape3d_label_rois -- input preprocessing on the device for a label map:
 * one read of the map gives, for every label 1..max_label, its bounding box
 * and voxel count, written as the entry of a device ROI table that crops the
 * map to the box and selects the label, ready for shape3d_batched_dev.  The
 * paper stages and transfers every input from the host and names this step
 * its open problem (Sec. 3, discussion of the results; Table 2, transfer
 * column); here the map stays in HBM and the table never leaves the device.
 *   labels:  DEVICE uint8, C-contiguous (dims[0], dims[1], dims[2]) label map
 *            (0 = background).
 *   dims, spacing: HOST, as shape3d.  spacing is copied into every entry.
 *   max_label: 1..255.  Voxels with larger labels are ignored.
 *   rois:    DEVICE shape3d_roi_ex[max_label], written: entry l - 1 has
 *            offset = the box's first voxel, dims = the box's extent,
 *            strides = the map's (dims[1] dims[2], dims[2]), label = l.  A
 *            label with no voxel gets a 1 x 1 x 1 crop at the origin, which
 *            then holds none of it (status SHAPE3D_EMPTY in the batch).  The
 *            entries also hold the boxes while they are built: their
 *            contents are defined once the call's work on `stream` is done.
 *   voxel_counts: DEVICE int64[max_label] (voxels per label) or NULL.
 *   max_dims: DEVICE int64[3] (the largest entry dims per axis, at least 1)
 *            or NULL.  The whole map's dims also bound every entry.
 * Enqueued on `stream` (no host synchronisation, no allocation).
 * Returns SHAPE3D_EINVAL for bad arguments (null pointers, max_label out of
 * range, buffers that are not device memory or are too small).
 */
int shape3d_label_rois(const uint8_t* labels, const int64_t dims[3], const double spacing[3], int32_t max_label,
                       shape3d_roi_ex* rois, int64_t* voxel_counts, int64_t* max_dims, void* stream);

/*
 * shape3d_noalloc -- shape3d_ex_async for callers that cannot allocate memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the call allocates nothing and needs no workspace argument.
 * Its scratch memory is a static device array of
 * SHAPE3D_NOALLOC_SCRATCH_BYTES (64 MiB) that each GPU the library runs on
 * holds until the process ends; the first call on a device (which must not be
 * under graph capture) looks its address up.
 *   vol, dtype, dims, spacing: as shape3d_ex; at most
 *           SHAPE3D_NOALLOC_MAX_VOXELS voxels, else SHAPE3D_ECAPACITY is
 *           returned and nothing is enqueued.
 *   out:    DEVICE double[6]; status: DEVICE int[1] (SHAPE3D_OK,
 *           SHAPE3D_EMPTY, or SHAPE3D_ECAPACITY when the mesh needs more
 *           vertex rows than the scratch holds, about 250,000 vertices; out
 *           is then untouched).
 * Asynchronous on `stream`.  Every call on one GPU uses that GPU's one
 * scratch array: calls that overlap on a device (other streams, other host
 * threads' streams) race and give undefined results; calls on one stream
 * are ordered and each starts from cleared counters.
 */
#define SHAPE3D_NOALLOC_SCRATCH_BYTES (64ull << 20)
#define SHAPE3D_NOALLOC_MAX_VOXELS (1ll << 24)
int shape3d_noalloc(const void* vol, int dtype, const int64_t dims[3], const double spacing[3], double* out,
                    int* status, void* stream);

/* Message describing the last failure of the calling thread ("" if none). */
const char* shape3d_last_error(void);

/* Frees the library's device workspace.  Safe to call at any time between calls. */
int shape3d_release(void);

/* Library version (major*100 + minor). */
int shape3d_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SHAPE3D_H */
