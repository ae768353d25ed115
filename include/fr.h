/*
 * fr.h -- C ABI of the MI355X radiomic spatial-mapping library
 * (libflashrad.so).
 *
 * The paper's problem statement ("Software design and extraction modes"):
 * the engine takes a medical image, a segmentation (VOI) mask and extraction
 * settings -- feature families, intensity discretisation, VOI handling and
 * mode -- and, in spatial-mapping mode, returns for every VOI voxel the
 * features of its local neighbourhood as maps aligned with the source
 * image.  The spatial benchmark set is Table 2's 93 maps: 18 first-order
 * ("statistics"), 24 GLCM, 16 GLRLM, 16 GLSZM, 14 GLDM (the paper's NGLDM)
 * and 5 NGTDM.  The feature definitions follow IBSI, to which the paper
 * defers ("IBSI compliance tests"); the readings fixed where the paper is
 * silent are listed beside each entry point.
 *
 * Conventions for every entry point
 *   - Volumes are C-ordered [nz][ny][nx], x fastest.  Linear index
 *     i = (z * ny + y) * nx + x.
 *   - "device" pointers are HIP device memory of the current device (for
 *     example torch tensors' data_ptr()); "host" pointers are CPU memory.
 *   - hip_stream is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued on it; results are valid once the stream has synchronised.
 *   - The caller owns every buffer it passes; the library keeps no pointer
 *     past the call.  The library owns a per-device scratch pool (level
 *     volume, compact index list, segment tables, a small parameter block,
 *     voxel-major map staging rows) that it grows on demand and reuses
 *     across calls; calls on one device share it, so they must be issued on
 *     one stream (or serialised) and not overlap from several host threads.
 *   - Argument errors found on the host are reported before any work is
 *     enqueued and leave every output untouched.  Errors that depend on the
 *     data (empty mask, more than 255 gray levels, n_mask mismatch) are found
 *     by the discretisation kernels on the device; every later kernel of the
 *     call then stops, so the outputs stay untouched.  fr_map enqueues
 *     without waiting and reports them through fr_map_status;
 *     fr_discretise and fr_map_matrices synchronise and return them.  A
 *     status < 0 is returned and fr_last_error() describes it
 *     (thread-local, valid until the next call from the same thread).  No
 *     C++ exception crosses this ABI.
 */
#ifndef FR_H_
#define FR_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fr_status;

enum {
  FR_OK = 0,
  FR_E_ARG = -1,         /* null pointer, non-positive size, bad enum, ... */
  FR_E_EMPTY_MASK = -2,  /* the mask holds no voxel                         */
  FR_E_RANGE = -3,       /* a value outside what the kernels support       */
  FR_E_NOMEM = -4,       /* scratch allocation failed                      */
  FR_E_DEVICE = -5,      /* a HIP call or kernel launch failed             */
  FR_E_CAPACITY = -6,    /* output buffer too small                        */
  FR_E_TIMEOUT = -7,     /* fr_server_wait: the job did not finish in time;
                            a served job not admitted by its deadline      */
  FR_E_CANCELLED = -8    /* a served job cancelled by fr_server_cancel      */
};

/* raw intensity types */
enum { FR_I16 = 1, FR_F32 = 2 };

/* discretisation: fixed bin width / fixed bin number (IBSI) */
enum { FR_FBW = 1, FR_FBN = 2 };

/* feature families (bit mask); maps are emitted in this family order */
enum {
  FR_FIRSTORDER = 1u << 0, /* 18 maps */
  FR_GLCM = 1u << 1,       /* 24 maps */
  FR_GLRLM = 1u << 2,      /* 16 maps */
  FR_GLSZM = 1u << 3,      /* 16 maps */
  FR_GLDM = 1u << 4,       /* 14 maps */
  FR_NGTDM = 1u << 5,      /*  5 maps */
  FR_ALL = 0x3Fu           /* 93 maps */
};

/* Largest kernel radius fr_map accepts (cube side 2r+1 <= 11); radii up to
 * 3 run on the fused fixed-radius kernels, 4 and 5 on the generic kernel. */
#define FR_MAX_RADIUS 5
/* Gray levels (Ng and the levels present in one neighbourhood) go up to 255. */
#define FR_MAX_LEVELS 255

/* Direction aggregation of the GLCM and GLRLM features (IBSI): merged
 * (matrices of the 13 directions summed, then features) or averaged
 * (features of each direction's matrix, then their mean). */
enum { FR_MERGED = 0, FR_AVERAGED = 1 };

/*
 * Extraction settings beyond fr_map's arguments (the paper's IBSI
 * configuration elements, "IBSI compliance tests": GLCM distance, NGLDM
 * coarseness and distance, direction aggregation).  fr_map uses the
 * defaults {1, 0, FR_MERGED, 0}.
 *   glcm_distance  1..2*FR_MAX_RADIUS: GLCM pairs (v, v + d * m) for the 13
 *                  direction representatives m
 *   gldm_alpha     0..254: a 26-neighbour u of v counts as dependent when
 *                  |g_u - g_v| <= alpha (the dependence distance stays 1)
 *   aggregation    FR_MERGED or FR_AVERAGED (GLCM and GLRLM; a direction
 *                  without any GLCM pair is left out of the GLCM mean, all
 *                  24 GLCM maps are NaN when no direction has one; GLRLM
 *                  counts Np = |V| per direction)
 *   reserved       0
 */
typedef struct fr_map_options {
  int32_t glcm_distance;
  int32_t gldm_alpha;
  int32_t aggregation;
  int32_t reserved;
} fr_map_options;

/*
 * fr_discretise -- intensity discretisation of the VOI (paper: settings of
 * "intensity discretization", done on the CPU in the paper's hybrid backend;
 * IBSI fixed bin number / fixed bin width).
 *
 *   FBN: g = floor(Ng * (X - Xmin) / (Xmax - Xmin)) + 1, capped at Ng;
 *        every g = 1 when Xmax == Xmin.  disc_value = Ng (integer 1..255).
 *   FBW: g = floor((X - Xlo) / w) + 1, at least 1 (values below a given
 *        lower bound take level 1), with w = disc_value > 0 and Xlo =
 *        disc_lower if finite, else Xmin; Ng = g(Xmax) <= 255.
 *   Xmin/Xmax are taken over all mask voxels.  Arithmetic is IEEE FP64
 *   (subtract, multiply, divide, floor; no contraction), so levels are
 *   bit-identical to any other FP64 evaluation of the same formula.
 *
 *   volume  device, dtype FR_I16 (int16) or FR_F32 (float32), [nz][ny][nx]
 *   mask    device, uint8 [nz][ny][nx], nonzero = inside the VOI
 *   levels  device, uint8 [nz][ny][nx] output, 0 outside the mask
 *   ng, xmin, xmax, n_mask   host outputs (any may be NULL)
 *
 * Synchronises hip_stream once to return the host outputs.
 * Errors: FR_E_ARG, FR_E_EMPTY_MASK, FR_E_RANGE (Ng > 255 or non-integer
 * bin count), FR_E_NOMEM, FR_E_DEVICE.  `levels` may have been written when
 * a data error is returned.
 */
fr_status fr_discretise(const void* volume, int32_t dtype, int32_t nx, int32_t ny,
                        int32_t nz, const uint8_t* mask, int32_t disc_mode,
                        double disc_value, double disc_lower, uint8_t* levels,
                        int32_t* ng, double* xmin, double* xmax, int64_t* n_mask,
                        void* hip_stream);

/* Number of maps fr_map emits for a family mask (93 for FR_ALL, 0 if the
 * mask holds unknown bits). */
int32_t fr_map_count(uint32_t families);

/* Name of map k (0-based, canonical order: family order above, then a fixed
 * feature order within each family), e.g. "glcm_JointEnergy"; NULL if k is
 * out of range.  Static storage. */
const char* fr_map_name(uint32_t families, int32_t k);

/*
 * fr_map -- spatial mapping (paper: "Software design and extraction modes";
 * the hot loop repeats the neighbourhood calculation for every VOI voxel,
 * Discussion).
 *
 * For every mask voxel c, in raster order (m = 0 .. n_mask-1), with
 *   V(c) = { u : |u - c|_inf <= kernel_radius, u inside the image, mask[u] },
 * the selected families' features of V(c) are written to
 *   out_maps[k * n_mask + m]   (float32, k = map index as fr_map_name).
 * Texture relations are restricted to V: GLCM over the 13 directions at
 * distance 1 (symmetric, merged); GLRLM maximal runs along the 13
 * directions (merged, Np = 13 |V|); GLSZM 26-connected zones; GLDM with
 * alpha = 0 (dependence = 1 + equal-level 26-neighbours in V); NGTDM over
 * the 26-neighbours in V of voxels that have at least one.  Non-finite
 * values mark undefined features (e.g. every GLCM map of a neighbourhood
 * without a voxel pair is NaN).  A dense map aligned with the image is the
 * caller's scatter of row k into the mask positions.
 *
 *   volume, mask   device, as fr_discretise
 *   spacing_mm     host, 3 doubles (sx, sy, sz) > 0; only TotalEnergy uses
 *                  them (voxel volume)
 *   kernel_radius  1..FR_MAX_RADIUS, in voxels (cube side 2r+1)
 *   families       non-empty subset of FR_ALL
 *   n_mask         number of nonzero mask bytes (checked on the device)
 *   out_maps       device float32 [fr_map_count(families)][n_mask]
 *   out_capacity_floats  size of out_maps in floats
 *
 * Asynchronous: everything is enqueued on hip_stream and the call returns
 * without waiting for the device.  The discretisation kernels (as
 * fr_discretise, into library scratch) check the mask count and Ng on the
 * device; the map kernels follow (a 32-level instance over every voxel,
 * then a 64-level one and a generic kernel for the neighbourhoods holding
 * more present levels, when Ng allows it; radii 4 and 5 use the generic
 * kernel alone), writing one 384-byte staging row per voxel, and a tile
 * transpose writes out_maps.  The library scratch is per device and grows
 * (after waiting for the device) when a larger job arrives: calls on one
 * device are issued on one stream, or they race on it.  Errors returned:
 * FR_E_ARG, FR_E_EMPTY_MASK
 * (n_mask <= 0), FR_E_RANGE (radius, families, bin count), FR_E_CAPACITY,
 * FR_E_NOMEM, FR_E_DEVICE; data errors are reported by fr_map_status.
 */
fr_status fr_map(const void* volume, int32_t dtype, int32_t nx, int32_t ny, int32_t nz,
                 const uint8_t* mask, const double* spacing_mm, int32_t disc_mode,
                 double disc_value, double disc_lower, int32_t kernel_radius,
                 uint32_t families, int64_t n_mask, float* out_maps,
                 int64_t out_capacity_floats, void* hip_stream);

/*
 * fr_map_ex -- fr_map with the IBSI extraction settings of fr_map_options
 * (NULL = the defaults, i.e. fr_map).  Non-default settings run on the
 * generic kernel.  Errors: those of fr_map, FR_E_RANGE / FR_E_ARG for an
 * option outside its range.
 */
fr_status fr_map_ex(const void* volume, int32_t dtype, int32_t nx, int32_t ny, int32_t nz,
                    const uint8_t* mask, const double* spacing_mm, int32_t disc_mode,
                    double disc_value, double disc_lower, int32_t kernel_radius,
                    uint32_t families, const fr_map_options* options, int64_t n_mask,
                    float* out_maps, int64_t out_capacity_floats, void* hip_stream);

/* Size of the fixed device scratch array of fr_map_noalloc (per device). */
#define FR_NOALLOC_SCRATCH_BYTES (64ull << 20)

/*
 * fr_map_noalloc -- fr_map for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, maps and errors as fr_map (default extraction
 * settings), enqueued the same way without waiting (fr_map_status reports
 * the device-side data checks), but it calls no hipMalloc, hipFree or
 * allocating routine: every buffer of the call (parameter block, segment
 * tables, level volume, mask-voxel list, overflow lists, staging rows when
 * they fit, a small generic-kernel region) lives in one static device array
 * of FR_NOALLOC_SCRATCH_BYTES that each device holds from its first call
 * until the process ends.  Jobs whose buffers exceed it return
 * FR_E_CAPACITY (roughly: 1 byte per volume voxel plus 20 bytes per mask
 * voxel, plus 384 bytes per mask voxel for coalesced output when that still
 * fits; more when more than 64 levels may share a neighbourhood).  Every
 * call on one device shares the array and leaves its contents for the next
 * call: calls that overlap on one device (on different streams or host
 * threads) race, so issue them on one stream.  The maps are bit-identical
 * to fr_map's.
 */
fr_status fr_map_noalloc(const void* volume, int32_t dtype, int32_t nx, int32_t ny, int32_t nz,
                         const uint8_t* mask, const double* spacing_mm, int32_t disc_mode,
                         double disc_value, double disc_lower, int32_t kernel_radius,
                         uint32_t families, int64_t n_mask, float* out_maps,
                         int64_t out_capacity_floats, void* hip_stream);

/*
 * fr_map_status -- synchronise hip_stream and report the data checks of the
 * most recent fr_map / fr_map_ex / fr_map_noalloc enqueued on the current
 * device (calls on
 * one device share one parameter block, so they are issued on one stream):
 * FR_OK (out_maps is valid), FR_E_EMPTY_MASK (no mask voxel), FR_E_ARG
 * (n_mask differs from the mask's count) or FR_E_RANGE (fixed bin width
 * giving more than 255 levels); *ng (may be NULL) receives the VOI Ng.
 * FR_E_ARG also when no map was enqueued on this device.
 */
fr_status fr_map_status(void* hip_stream, int32_t* ng);

/*
 * fr_map_matrices -- the integer texture matrices the map kernel counts for
 * a sample of mask voxels, for bit-exact comparison with any other
 * implementation of the definitions above.  Runs the same kernel as fr_map
 * (same counting code), restricted to the sample, and expands its compact
 * per-neighbourhood tables to dense tables over the VOI levels 1..Ng
 * (row a = level a+1).  Also writes the sample's maps like fr_map, with
 * n_sample in place of n_mask.  Only the tables of the selected families
 * are counted (the others stay zero; the level histogram is always filled).
 * A sample index outside 0..n_mask-1 yields NaN maps and zero tables.
 * Synchronous (it checks Ng before the tables are written).  options: as
 * fr_map_ex (NULL = defaults); the tables are then the ones those settings
 * count (GLDM with alpha, the GLCM at the distance; averaged aggregation
 * dumps the sum of the direction matrices).
 *
 *   sample      device int64 [n_sample], compact mask indices (0..n_mask-1)
 *   ng_expected the VOI Ng (from fr_discretise); checked
 *   glcm        device int32 [n_sample][ng][ng]        co-occurrence counts
 *   glrlm       device int32 [n_sample][ng][2r+1]      col j-1: run length j
 *   glszm       device int32 [n_sample][ng][(2r+1)^3]  col s-1: zone size s
 *   gldm        device int32 [n_sample][ng][27]        col k-1: dependence k
 *   ngtdm_n     device int32 [n_sample][ng]            voxel counts n_i
 *   ngtdm_S     device int64 [n_sample][ng]   s_i * lcm(1..26), exact
 *   hist        device int32 [n_sample][ng]            level histogram
 *   out_maps    device float32 [fr_map_count(families)][n_sample]
 * The matrix buffers are overwritten entirely.  Same errors as fr_map.
 */
fr_status fr_map_matrices(const void* volume, int32_t dtype, int32_t nx, int32_t ny,
                          int32_t nz, const uint8_t* mask, const double* spacing_mm,
                          int32_t disc_mode, double disc_value, double disc_lower,
                          int32_t kernel_radius, uint32_t families,
                          const fr_map_options* options, int64_t n_mask,
                          const int64_t* sample, int64_t n_sample, int32_t ng_expected,
                          int32_t* glcm, int32_t* glrlm, int32_t* glszm, int32_t* gldm,
                          int32_t* ngtdm_n, int64_t* ngtdm_S, int32_t* hist,
                          float* out_maps, void* hip_stream);

/*
 * fr_scalar -- whole-VOI features (paper: the scalar extraction mode of
 * "Software design and extraction modes"; the paper measured the CPU faster
 * than its GPU backend for scalar extraction, so this runs on the host).
 * The definitions are fr_map's with the neighbourhood taken to be the whole
 * mask, V = {u : mask[u]}: a map value at a voxel whose cube covers the VOI
 * equals the scalar value.  Matrices are counted exactly; features in FP64.
 *
 *   volume, mask   HOST memory, layout as fr_discretise
 *   spacing_mm     host, 3 doubles > 0
 *   disc_*         as fr_discretise (FBW: Ng = level of the VOI maximum)
 *   families       non-empty subset of FR_ALL
 *   out            host double [fr_map_count(families)], order of fr_map_name
 *   out_capacity   size of out in doubles
 * Synchronous; no device work.  Errors: FR_E_ARG, FR_E_EMPTY_MASK,
 * FR_E_RANGE, FR_E_CAPACITY (message in fr_last_error).
 */
fr_status fr_scalar(const void* volume, int32_t dtype, int32_t nx, int32_t ny, int32_t nz,
                    const uint8_t* mask, const double* spacing_mm, int32_t disc_mode,
                    double disc_value, double disc_lower, uint32_t families, double* out,
                    int32_t out_capacity);

/* The same message as fr_last_error() (kept for callers of this family). */
const char* fr_scalar_last_error(void);

/*
 * Batched spatial mapping -- many VOIs (different sizes, radii, bin counts,
 * raw types) mapped by one enqueue.  The paper runs one VOI per call and
 * names batching across many VOIs as the route to throughput for studies of
 * many patients (Discussion); the features of each job are exactly those of
 * fr_map on the same inputs (same kernels' arithmetic, bit-identical maps).
 *
 * One fr_job describes one VOI with fr_map's arguments (same meaning, same
 * layout, same device-pointer rules).  The caller keeps every buffer a job
 * names alive and unmoved from fr_batch_prepare until the batch is prepared
 * again or destroyed; the volumes may be rewritten between launches (the
 * next launch maps the new values with the prepared settings).
 */
typedef struct fr_job {
  const void* volume;          /* device, dtype FR_I16 / FR_F32, [nz][ny][nx] */
  const uint8_t* mask;         /* device, uint8 [nz][ny][nx]                  */
  float* out_maps;             /* device float32 [fr_map_count(families)][n_mask] */
  int64_t out_capacity_floats; /* size of out_maps in floats                  */
  int64_t n_mask;              /* nonzero mask bytes (checked on the device)  */
  double spacing_mm[3];        /* (sx, sy, sz) > 0                            */
  double disc_value;           /* FBW bin width / FBN bin count               */
  double disc_lower;           /* FBW lower bound, NaN = VOI minimum          */
  int32_t dtype, nx, ny, nz;
  int32_t disc_mode;           /* FR_FBW / FR_FBN                             */
  int32_t kernel_radius;       /* 1..FR_MAX_RADIUS                            */
  uint32_t families;           /* non-empty subset of FR_ALL                  */
  int32_t reserved;            /* set to 0                                    */
} fr_job;

typedef struct fr_batch_s* fr_batch;

/* Create an empty batch on the current device. */
fr_status fr_batch_create(fr_batch* out);

/* Release a batch, its device workspace and its captured graph (NULL ok).
 * Work enqueued by fr_batch_launch must have completed. */
fr_status fr_batch_destroy(fr_batch b);

/*
 * fr_batch_prepare -- validate n_jobs jobs on the host (every fr_map argument
 * check except those that need the data) and plan the batch: one
 * discretisation segment table over all volumes, and for each variant
 * present (raw type, radius, level class: at most 32 or up to 255 present
 * levels per neighbourhood, from Ng and the cube size) a table of work
 * items (job, first voxel).  Allocates the batch's device workspace: level
 * volumes (1 B/voxel), mask-voxel lists (4 B/mask voxel), staging rows
 * (384 B/mask voxel), two overflow lists per variant (8 B/mask voxel each),
 * segment and item tables, and generic-kernel scratch when a job may hold
 * more than 64 levels or uses a radius above 3.  Synchronous (uploads the
 * tables); replaces any previous plan and graph, so work enqueued by an
 * earlier fr_batch_launch of this batch must have completed.  The jobs
 * array is copied.
 * Errors: FR_E_ARG, FR_E_RANGE, FR_E_CAPACITY (with the job index in
 * fr_last_error), FR_E_NOMEM, FR_E_DEVICE.
 */
fr_status fr_batch_prepare(fr_batch b, const fr_job* jobs, int32_t n_jobs);

/*
 * fr_batch_launch -- enqueue the whole batch on hip_stream: batched
 * discretisation (3 launches); per raw type one fused persistent map pass
 * over the work items of every job of radius 1..3 (one kernel for all
 * three radii, items taken from a device work queue, largest estimated
 * work first; 32 present levels, MCC problems stashed), the MCC kernel over
 * the stash, per raw type one fused pass of the 64-level instances over
 * the neighbourhoods the first pass handed on, the generic kernel over the
 * neighbourhoods with more than 64 present levels (and over every voxel of
 * a radius above 3), and a batched transpose into every job's out_maps.
 * All on hip_stream; no host synchronisation and no allocation.  With
 * use_graph != 0 the sequence is captured into a HIP graph on the first
 * call (hip_stream must then be non-NULL) and the graph is replayed on
 * later calls.  A job that fails a data check on the device (mask count !=
 * n_mask, FBW Ng > 255) is skipped and its out_maps left untouched; the
 * other jobs are mapped.  Errors: FR_E_ARG, FR_E_DEVICE.
 */
fr_status fr_batch_launch(fr_batch b, void* hip_stream, int32_t use_graph);

/*
 * fr_batch_status -- synchronise hip_stream and report the last launch's
 * per-job outcome: job_status[j] = FR_OK, FR_E_EMPTY_MASK, FR_E_ARG (mask
 * count != n_mask) or FR_E_RANGE (FBW Ng > 255); ng[j] = the
 * job's VOI Ng.  Either array may be NULL (else n_jobs entries, host).
 * Returns FR_E_RANGE if any job failed, else FR_OK.
 */
fr_status fr_batch_status(fr_batch b, int32_t* job_status, int32_t* ng, void* hip_stream);

/*
 * fr_batch_autotune -- on the prepared batch, time each variant's (raw type,
 * radius, level class) fused first pass and MCC kernel over work-item sizes
 * {2, 4, 8, 16} voxels.  Keeps the fastest for this batch and as the
 * default of later batches (and served jobs) of this process.  The maps do
 * not depend on the choice (it orders work only).  Runs the batch (its
 * outputs are valid afterwards) and synchronises hip_stream.  Errors:
 * FR_E_ARG, FR_E_DEVICE.
 */
fr_status fr_batch_autotune(fr_batch b, void* hip_stream);

/*
 * fr_batch_describe -- the plan: *n_variants, and for each variant 8 int32
 * in table (host, table_len entries): dtype, radius, bound of the present
 * levels (largest min(Ng, cube) of its jobs), jobs, work items, voxels per
 * item, grid of its pass, local levels of the first pass's instance (32;
 * 0: generic).
 */
fr_status fr_batch_describe(fr_batch b, int32_t* n_variants, int32_t* table, int32_t table_len);

/* The same message as fr_last_error() (kept for callers of this family). */
const char* fr_batch_last_error(void);

/*
 * Served spatial mapping -- a continuous-batching request loop for map jobs
 * that arrive over time (many patients' VOIs submitted while others are
 * being mapped; the paper's Discussion names batching across VOIs as the
 * route to throughput).  Each job's maps are exactly those of fr_map on the
 * same inputs (same kernels; bit-identical whatever runs beside it).
 *
 * The server allocates one device arena of hbm_budget_bytes at creation and
 * nothing afterwards.  A job's footprint (fr_server_footprint) is one arena
 * block holding its map-major output (4 B per map and mask voxel) and its
 * working buffers: copies of its raw volume and mask, its level volume (1 B
 * per voxel), mask-voxel list (4 B per mask voxel), staging rows (384 B per
 * mask voxel) and small tables.  The working buffers return to the arena when the job ends;
 * the output part stays until fr_server_release.  A
 * worker thread admits queued jobs when one of `slots` HIP streams is free
 * and a block of the job's footprint is free in the arena (the arena size is
 * the HBM budget admission runs against), enqueues the job's pipeline
 * (copies, discretisation, map kernel, transpose, status read-back) on that
 * stream without a host synchronisation, and retires it when the stream's
 * event completes.  Jobs on different slots overlap on the device.  Outputs
 * stay in the arena until fr_server_release.  Times are CLOCK_MONOTONIC
 * seconds.
 *
 * Admission order: submission order, except that when the oldest queued job
 * (the head) does not fit, a later job that fits may pass it -- at most
 * max_bypass jobs per head, after which nothing passes it until it is
 * admitted (so a large job waits for at most max_bypass extra jobs).  A job
 * still queued at its deadline (fr_server_submit_ex) is dropped with
 * FR_E_TIMEOUT; a cancelled job (fr_server_cancel) ends with
 * FR_E_CANCELLED.  Neither changes any other job's maps.  The same policy
 * can be replayed on the host in virtual time (fr_admission_replay).
 */
typedef struct fr_server_s* fr_server;

typedef struct fr_server_config {
  int64_t hbm_budget_bytes; /* arena size (>= 1 MiB)                        */
  int32_t slots;            /* concurrent jobs / streams, 1..16             */
  int32_t max_bypass;       /* later jobs that may pass a head job that does
                               not fit, 0..1024 (0: strict submission order) */
} fr_server_config;

typedef struct fr_result {
  const float* maps;        /* device [count][n_mask] in the arena; NULL unless
                               done with status FR_OK; valid until release  */
  int64_t n_mask;
  int64_t footprint_bytes;
  double t_submit, t_admit, t_done;
  int32_t done;             /* 1 once the job has finished                  */
  int32_t status;           /* FR_OK, or the job's device-side error        */
  int32_t ng;               /* VOI gray-level count                         */
  int32_t count;            /* number of maps                               */
} fr_result;

typedef struct fr_server_info {
  int64_t submitted, completed, failed, mapped_voxels;
  int64_t arena_bytes, arena_used_bytes, arena_peak_bytes;
  double p50_ms, p99_ms, mean_ms; /* submit-to-done latency, nearest rank   */
  int32_t slots, max_inflight, queued, inflight;
} fr_server_info;

/* Create a server on the current device (allocates the arena, the slot
 * streams and a worker thread).  Errors: FR_E_ARG, FR_E_NOMEM, FR_E_DEVICE. */
fr_status fr_server_create(const fr_server_config* cfg, fr_server* out);

/* Arena bytes a job would take (validates the job like fr_server_submit). */
fr_status fr_server_footprint(const fr_job* job, int64_t* bytes);

/*
 * Queue a job; returns at once with a ticket.  The job is an fr_job whose
 * out_maps is NULL and out_capacity_floats 0 (the output lives in the
 * arena).  volume and mask may be device or host memory; they are copied
 * into the arena at admission, so they must stay valid and unchanged (and
 * any device work writing them must have completed) until the job is
 * reported done.  Errors (host checks, nothing queued): FR_E_ARG,
 * FR_E_RANGE, FR_E_CAPACITY (footprint larger than the whole arena).
 */
fr_status fr_server_submit(fr_server s, const fr_job* job, int64_t* ticket);

/* Per-job submission options. */
typedef struct fr_submit_options {
  double deadline_ms;       /* > 0: drop the job with FR_E_TIMEOUT if it is not
                               admitted within this many ms of submission
                               (a job already running always completes);
                               0: no deadline                               */
  int32_t reserved[2];      /* set to 0                                     */
} fr_submit_options;

/* fr_server_submit with options (NULL = none).  Errors: those of
 * fr_server_submit, FR_E_ARG for a negative deadline or nonzero reserved. */
fr_status fr_server_submit_ex(fr_server s, const fr_job* job, const fr_submit_options* options,
                              int64_t* ticket);

/*
 * Cancel a job.  A queued job ends at once with status FR_E_CANCELLED and
 * never runs; a running job's kernels complete (they cannot be stopped), its
 * block is freed as soon as they have, and it ends with FR_E_CANCELLED and
 * no maps.  Either way the ticket still needs fr_server_release.  Errors:
 * FR_E_ARG (unknown ticket, or the job had already finished).
 */
fr_status fr_server_cancel(fr_server s, int64_t ticket);

/*
 * Failure injection for tests of the admission path: the next `n` jobs the
 * server would admit fail instead as if the allocation of their arena block
 * had failed (status FR_E_NOMEM, nothing enqueued, no block kept); admission
 * then goes on with the following jobs.  n = 0 clears it.  Errors: FR_E_ARG.
 */
fr_status fr_server_inject_alloc_failures(fr_server s, int32_t n);

/* Tickets finished since the previous poll and not yet released, oldest
 * first (at most max_tickets; the rest stay for the next poll). */
fr_status fr_server_poll(fr_server s, int64_t* tickets, int32_t max_tickets, int32_t* n_done);

/* Block until the job has finished; timeout_ms < 0 waits without limit.
 * Errors: FR_E_ARG (unknown ticket), FR_E_TIMEOUT. */
fr_status fr_server_wait(fr_server s, int64_t ticket, double timeout_ms);

/* State, status, output and timestamps of a job (host struct). */
fr_status fr_server_result(fr_server s, int64_t ticket, fr_result* r);

/* Copy a finished job's maps ([count][n_mask] float32) to dst (device or
 * host memory of capacity_floats floats), enqueued on hip_stream.  The
 * ticket must not be released before the copy has completed.  Errors:
 * FR_E_ARG (unknown, unfinished or failed job), FR_E_CAPACITY, FR_E_DEVICE. */
fr_status fr_server_copy(fr_server s, int64_t ticket, float* dst, int64_t capacity_floats,
                         void* hip_stream);

/* Free a finished job's arena block (its maps pointer becomes invalid) and
 * forget the ticket.  Errors: FR_E_ARG (unknown or unfinished ticket). */
fr_status fr_server_release(fr_server s, int64_t ticket);

/* Counters and latency percentiles over every finished job. */
fr_status fr_server_stats(fr_server s, fr_server_info* out);

/* Drop queued jobs, wait for running ones, free everything.  No other call
 * on this server may run concurrently or follow. */
fr_status fr_server_destroy(fr_server s);

/* The same message as fr_last_error() (kept for callers of this family). */
const char* fr_server_last_error(void);

/*
 * fr_admission_replay -- the server's admission policy (arena first fit,
 * bounded bypass, deadlines, cancellation, injected allocation failures)
 * run on the host in virtual time over a scripted event list, with a
 * virtual HBM budget and no device: for tests and capacity planning.
 * Events are applied in order (t non-decreasing); after each one the
 * policy admits what it can at time t.  Each outcome appends one record.
 */
enum {
  FR_ADMIT_SUBMIT = 0,     /* a job of `bytes` (footprint) arrives          */
  FR_ADMIT_CANCEL = 1,     /* cancel job `ticket` (queued: dropped at once;
                              running: it ends cancelled at its COMPLETE)   */
  FR_ADMIT_COMPLETE = 2,   /* running job `ticket` finishes: frees its slot
                              and its block                                */
  FR_ADMIT_FAIL_NEXT = 3   /* the next `value` admissions fail             */
};
enum {
  FR_ADMITTED = 0,         /* admitted at `offset` of the arena             */
  FR_ADMIT_EXPIRED = 1,    /* deadline passed while queued                  */
  FR_ADMIT_CANCELLED = 2,  /* cancelled while queued                        */
  FR_ADMIT_ALLOC_FAILED = 3, /* admission failed by injection               */
  FR_ADMIT_REJECTED = 4    /* footprint larger than the whole budget        */
};
typedef struct fr_admit_event {
  double t;                /* virtual time, seconds                         */
  double deadline_ms;      /* SUBMIT: as fr_submit_options (0: none)        */
  int64_t ticket;          /* SUBMIT: a new id; CANCEL, COMPLETE: a job's   */
  int64_t bytes;           /* SUBMIT: footprint                             */
  int32_t kind;            /* FR_ADMIT_SUBMIT ...                           */
  int32_t value;           /* FAIL_NEXT: count                              */
} fr_admit_event;
typedef struct fr_admit_record {
  double t;                /* time of the event that produced it            */
  int64_t ticket;
  int64_t offset;          /* FR_ADMITTED: block offset, else -1            */
  int32_t outcome;         /* FR_ADMITTED ...                               */
  int32_t reserved;
} fr_admit_record;
/* Errors: FR_E_ARG (bad arguments, unknown or repeated ticket, time going
 * back, COMPLETE of a job that is not running), FR_E_CAPACITY (more than
 * max_records records). */
fr_status fr_admission_replay(int64_t budget_bytes, int32_t slots, int32_t max_bypass,
                              const fr_admit_event* events, int32_t n_events,
                              fr_admit_record* records, int32_t max_records, int32_t* n_records);

/*
 * Kernel timing for measurement: when enabled, fr_map records a pair of HIP
 * events on its stream around the map kernel.  fr_profile_read() waits for
 * the recorded launches, returns the summed map-kernel time in ms and the
 * number of launches since the previous read, and resets both.
 */
fr_status fr_profile_enable(int32_t enable);
fr_status fr_profile_read(double* map_kernel_ms, int64_t* launches);

/*
 * The one error message of this ABI: that of the calling thread's last
 * failing call to any entry point (map, batch, server, scalar), "" after a
 * call that succeeded.  Thread-local, valid until the next call from the
 * same thread.
 */
const char* fr_last_error(void);

/* Library version string. */
const char* fr_version(void);

/*
 * Identity of the sources this library was built from: the first 16 hex
 * digits of a SHA-256 over the library's source files (the build computes
 * it and compiles it in; "unknown" for a build that did not).  A caller
 * that holds the sources can recompute it to check that the library is
 * not stale.  Static storage; never fails.
 */
const char* fr_source_hash(void);

#ifdef __cplusplus
}
#endif

#endif /* FR_H_ */
