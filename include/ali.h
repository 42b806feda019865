/*
 * ali.h -- C ABI of the MI355X travel-time solver for generally anisotropic media
 * (ALI-FMM: Ludlam, Tant, Dolean, Curtis, arXiv 2302.10988).
 *
 * What it computes (paper Section 2, eq. 1): first-arrival qP travel times from a point
 * source to every node of a square 2-D grid, in a medium given per node by a material
 * (stiffness tensor and density, Section 3.2) and the orientation of its symmetry axis.
 * Each node value is the paper's locally interpolated wavefront estimate (Sections
 * 4.1-4.3) from already-known diamond neighbours; the GPU reaches the same discrete fixed
 * point as the paper's heap-ordered Fast Marching by a tiled data-parallel relaxation.
 *
 * Conventions for every entry point:
 *   - nodes (i, j): i = x column 0..nx-1, j = z row 0..nz-1 (z = depth, downward);
 *     spacing h [m]; fields are row-major [nz][nx], float32 unless the name ends in _f64.
 *   - orientation [rad]: angle of the symmetry axis measured from +x toward +z.  The
 *     paper's velocity-curve angle is measured from the perpendicular (c22) axis; only the
 *     difference matters and any multiple of pi is harmless (180-degree symmetry).
 *   - material stiffness [Pa] is given in the axis frame: "3" = symmetry axis, "1" = the
 *     in-plane direction across it.  The qP speed uses c11, c13, c33, c55 (the paper's
 *     c22, c23, c33, c44 of its YZ plane); c44, c66 are carried for shear modes.
 *   - travel times in seconds; +INFINITY marks a node the wave cannot reach.
 *   - pointers named d_* are device pointers (caller-owned, on the handle's device);
 *     the others are host pointers.  Calls are asynchronous on the handle's stream
 *     unless stated; a stats struct is filled before the call returns.
 *   - errors: every function returns ali_status; nothing throws across the ABI.  Invalid
 *     arguments return ALI_EINVAL before any device work is queued; the message is
 *     available from ali_last_error(handle).
 */
#ifndef ALI_H
#define ALI_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ALI_OK = 0,
    ALI_EINVAL = -1,        /* invalid argument (sizes, material, source, orientation)   */
    ALI_ENOMEM = -2,        /* device allocation for the handle's scratch failed          */
    ALI_EDEVICE = -3,       /* a HIP call failed                                           */
    ALI_ENOCONV = -4,       /* relaxation hit max_sweeps; T holds the last iterate         */
    ALI_EUNSUPPORTED = -5
} ali_status;

typedef struct { int32_t nx, nz; double h; } ali_grid;

typedef struct { double c11, c13, c33, c55, c44, c66, rho; } ali_material;

typedef struct { int32_t i, j; } ali_node;

typedef struct {
    int32_t src_box_radius;  /* straight-ray box half-width in nodes (Section 4.4); default 2   */
    int32_t max_sweeps;      /* cap on outer relaxation passes; default 1000000                 */
    int32_t inner_sweeps;    /* cap on sweeps inside one tile visit (unfinished nodes carry over
                                to the next pass); default 2                                    */
    int32_t band_cells;      /* width of the relaxation time band in node spacings at the
                                fastest phase speed; 0 = no band; default 1                   */
    int32_t ray_window;      /* ray tracer: candidate window either side of the straight-ahead
                                intersection, in node spacings (Section 5.1 limits the candidates,
                                no value given); default 4                                      */
    int32_t ray_max_pts;     /* ray tracer: maximum points per path; default 4096                */
    int32_t arith;           /* float32 entry points: ALI_ARITH_MIXED (default), _F32 or _F64     */
    int32_t ray_sub;         /* ray tracer: candidates per node spacing along a plane (the paper's
                                finer subgrid); ray_window * ray_sub <= 32; default 8             */
    int32_t graph;           /* 1: relaxation passes are replayed from captured HIP graphs (one
                                per argument signature, kept by the handle); 0: launched one by
                                one; default 1                                                 */
    int32_t wave;            /* ALI_WAVE_QP (default): the in-plane quasi-P wave of the paper;
                                ALI_WAVE_SH: the shear wave polarised normal to the plane       */
    int32_t ray_planes;      /* ray tracer plane families: ALI_RAY_CHANGING (default) or a fixed
                                family / the fastest of the four fixed families (below)         */
    int32_t velocity;        /* ALI_VEL_CHRISTOFFEL (default) or ALI_VEL_TABLE (below)           */
    const float* d_node_A;   /* per-node stiffness / density (device, caller-owned), NULL (default)
                                = the material table.  Otherwise [nodes][4] float32: A11, A13, A33,
                                A55 of every node in m^2/s^2 (A = C / rho, the layout of the
                                stiffness gradient), nodes in the order of d_mat_id (for a batch,
                                the media's nodes concatenated as there).  Each node needs finite
                                A11, A33, A55 > 0 and A11 A33 > A13^2, else ALI_EINVAL after the
                                device check.  The qP forward solves (single medium, batch, nested
                                source grids and subgrid: fine nodes take the nearest node's) and
                                the adjoint and misfit gradients take it; ray tracing, SH and the
                                velocity table return ALI_EUNSUPPORTED.
                                The material table and ids must still be valid; they are then not
                                read for the speeds.                                           */
    int32_t persistent;      /* 1: every relaxation pass of a forward solve runs in one cooperative
                                launch (all work-groups resident, grid barriers between the
                                scheduling and relaxation phases of a pass, every barrier wait
                                bounded: a wait past 5 s returns ALI_EDEVICE); 0 (default): one
                                scheduling and one relaxation launch per pass, replayed from
                                captured graphs.  Both reach the same fields bit for bit.  The
                                cooperative launch needs the device's cooperative-launch
                                resources: while another process holds them (one that has made
                                such a launch) the runtime refuses it and the call returns
                                ALI_EDEVICE, naming the refused launch in ali_last_error.      */
    int32_t visit_tiles;     /* most tiles one wave visits at once in a pass with more tiles than
                                resident waves (their marked nodes share 64-lane chunks): 1..4,
                                0 (default) = 4.  The fields do not depend on it.              */
    int32_t adjoint_band_cells;    /* band of the adjoint relaxation in node spacings at the fastest
                                      phase speed; 0 (default) = band_cells                    */
    int32_t adjoint_inner_sweeps;  /* sweep cap of an adjoint tile visit; 0 (default) =
                                      inner_sweeps.  The gradient does not depend on either.   */
} ali_options;

/* Speeds of the solve (Section 3.2).  CHRISTOFFEL: the phase speed of every stencil and the
   group speed of every straight ray solved at run time.  TABLE: the paper's cheaper
   variant: per material, the exact phase speeds at whole degrees (0..90) of the angle
   between the wavefront normal and the symmetry axis and the exact group speeds at whole
   degrees of the group angle, linearly interpolated (tables built on the device at the
   start of each call).  Forward solves, nested source grids and rays take either; the
   adjoint entry points need CHRISTOFFEL (ALI_EUNSUPPORTED otherwise). */
enum { ALI_VEL_CHRISTOFFEL = 0, ALI_VEL_TABLE = 1 };

/* Plane families of the ray tracer (Section 5.1).  CHANGING: each step uses the family at
   the largest angle to the last segment, candidates around the straight-ahead point, and
   stops within 1.6 spacings of the source.  FIXED_*: one family for the whole ray
   (x = k, z = k, x + z = k, x - z = k), its planes strictly between the receiver and the
   source crossed in order; on each plane every grid node is costed first, then the fine
   window (ray_window, ray_sub) around the best node; the last point joins the source.
   FASTEST_FIXED: the four fixed families, the fastest reached ray kept. */
enum { ALI_RAY_CHANGING = 0, ALI_RAY_FIXED_X = 1, ALI_RAY_FIXED_Z = 2, ALI_RAY_FIXED_DIAG = 3,
       ALI_RAY_FIXED_ANTI = 4, ALI_RAY_FASTEST_FIXED = 5 };

/* Wave of a call.  QP uses c11, c13, c33, c55 (needs c11, c33, c55 > 0 and
   c11*c33 > c13^2).  SH (an extension the paper names in Section 6) uses c44 and c66: its
   Christoffel entry is c66 n1^2 + c44 n3^2 (n1 across the axis, n3 along it), an
   elliptical slowness curve (needs c44, c66 > 0).  The SH speeds are those of the qP wave
   of the record c11 = c66, c33 = c44, c55 = min(c44, c66), c13 = -c55, whose in-plane
   Christoffel matrix is diagonal with the SH entry as its larger one, so every kernel runs
   unchanged on that record.  Rays and the orientation gradient follow the same speeds;
   the stiffness gradient is qP only. */
enum { ALI_WAVE_QP = 0, ALI_WAVE_SH = 1 };

/* Arithmetic of the float32 entry points.  MIXED keeps travel times, scores and every
   comparison that decides a stencil in float64 and computes each stencil's wavefront /
   phase-speed increment in float32 (within a few 1e-7 of the float64 oracle on the
   straight-ray box; the nested source grids compute MIXED in float64, see
   ali_solve_traveltime_refined); F32 does everything in float32: fastest, and outside the
   1e-4 bar (stencil choices near score ties follow the float32 rounding of the stored
   times: 1.7e-4 on the 512 x 512 weld); F64 does everything in float64.  Output is
   float32 in all three. */
enum { ALI_ARITH_MIXED = 0, ALI_ARITH_F32 = 1, ALI_ARITH_F64 = 2 };

typedef struct {
    int64_t node_updates;    /* evaluations of the local update at a non-fixed node          */
    int64_t stencil_evals;   /* single-stencil estimates computed inside those updates        */
    int64_t tile_visits;     /* tile passes of the relaxation                                */
    int64_t nodes;           /* grid nodes times fields                                       */
    int32_t outer_iters;     /* outer relaxation passes (= relaxation kernel launches)        */
    int32_t converged;       /* 1 if every field reached a bitwise fixed point                */
    double  ms;              /* time of the whole call on the stream (HIP events)             */
    double  relax_ms;        /* summed duration of the relaxation kernel launches (HIP events) */
} ali_solve_stats;

/* One medium of a batch.  Offsets count elements of the arrays the batch calls take. */
typedef struct {
    ali_grid grid;
    int32_t mat_offset, n_mats;   /* this medium's materials: mats[mat_offset .. + n_mats); its
                                     material ids index this range                            */
    int64_t node_offset;          /* first node of this medium's [nz][nx] arrays (material ids,
                                     orientation, gradient)                                    */
    int32_t src_offset, n_src;    /* this medium's sources: srcs[src_offset .. + n_src)          */
    int32_t rec_offset, n_rec;    /* this medium's receivers: recv[rec_offset .. + n_rec)
                                     (gradient calls; ignored by ali_solve_batch)             */
} ali_medium;

typedef struct ali_handle ali_handle;

/* Create a handle bound to HIP device `device` and stream `hip_stream` (a hipStream_t;
   NULL = the default stream).  The handle owns its scratch memory (tile lists, flags,
   per-node constants), grown on demand and freed by ali_destroy.  One handle must not be
   used from two threads at once. */
ali_status ali_create(ali_handle** out, int device, void* hip_stream);
ali_status ali_destroy(ali_handle* h);
ali_status ali_set_stream(ali_handle* h, void* hip_stream);
void ali_default_options(ali_options* opt);
/* How long a grid barrier of the persistent relaxation (ali_options.persistent) waits for
   the other work-groups before the call gives up with ALI_EDEVICE (default 5 s; seconds
   >= 0; a wait is also cut short once any work-group has given up). */
ali_status ali_set_barrier_timeout(ali_handle* h, double seconds);
const char* ali_status_string(ali_status s);
const char* ali_last_error(const ali_handle* h);

/* Travel-time fields for n_src point sources in one medium (paper Sections 2 and 4),
   solved together in one batched relaxation.
     grid           nx, nz >= 3, h > 0
     mats[n_mats]   1 <= n_mats <= 256; each needs rho > 0, c11, c33, c55 > 0 and
                    c11*c33 > c13^2 (in-plane positive definiteness)
     d_mat_id       [nz][nx] uint8 material index (< n_mats)
     d_orient       [nz][nx] float32 symmetry-axis angle [rad], finite
     srcs[n_src]    source nodes (host array), inside the grid
     d_T            [n_src][nz][nx] float32 output
   Node values inside the source box come from straight rays at the group speed of the
   source node's material (Section 4.4, first paragraph); every other value is the ALI
   local estimate (Sections 4.1-4.3) at the unique fixed point of the update.
   A NaN/inf orientation is reported as ALI_EINVAL after the device check.
   If stats != NULL the call synchronises the stream and fills it. */
ali_status ali_solve_traveltime(ali_handle* h, const ali_grid* grid,
                                const ali_material* mats, int32_t n_mats,
                                const uint8_t* d_mat_id, const float* d_orient,
                                const ali_node* srcs, int32_t n_src,
                                const ali_options* opt, float* d_T,
                                ali_solve_stats* stats);

/* Same computation in float64 (orientation and output in double): the logic-parity
   mode used to compare with a double-precision reference. */
ali_status ali_solve_traveltime_f64(ali_handle* h, const ali_grid* grid,
                                    const ali_material* mats, int32_t n_mats,
                                    const uint8_t* d_mat_id, const double* d_orient,
                                    const ali_node* srcs, int32_t n_src,
                                    const ali_options* opt, double* d_T,
                                    ali_solve_stats* stats);

/* Allocation-free variant of ali_solve_traveltime, for callers that cannot allocate device
   memory: code under HIP graph capture, tight serving loops, harnesses that forbid
   allocation.  Same arguments, computation, options, output and errors; every scratch
   buffer is carved from one static device array of ALI_NOALLOC_SCRATCH_BYTES per device
   (file scope in the library, held until the process ends), so the call makes no
   hipMalloc or hipFree and calls no allocating library routine.  Passes are launched one
   by one (opt->graph is ignored).  In the default mixed arithmetic a solve needs about
   64 B per node plus 9 B per node and source (a 512 x 512 medium takes up to 21 sources);
   a larger one returns ALI_EINVAL before any device work, with the needed size in
   ali_last_error.  Every call on a device shares that device's array and it keeps the
   last call's contents (each call clears what must start at zero): calls that overlap on
   one device (two handles, threads or streams) race and must be serialised by the caller. */
#define ALI_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
ali_status ali_solve_traveltime_noalloc(ali_handle* h, const ali_grid* grid,
                                        const ali_material* mats, int32_t n_mats,
                                        const uint8_t* d_mat_id, const float* d_orient,
                                        const ali_node* srcs, int32_t n_src,
                                        const ali_options* opt, float* d_T,
                                        ali_solve_stats* stats);

/* ---- nested fine grids around the source (paper Section 4.4) ------------------------- */

#define ALI_MAX_LEVELS 8
typedef struct {
    int32_t n_levels;                  /* fine grids, finest first; 0 .. ALI_MAX_LEVELS       */
    int32_t density[ALI_MAX_LEVELS];   /* nodes per grid spacing: odd, 3 .. 255, each divisible
                                          by the next                                          */
    int32_t radius[ALI_MAX_LEVELS];    /* the grid is used until the front passes this Chebyshev
                                          radius around the source [cells]; non-decreasing    */
    double start_half_width;           /* straight rays on the finest grid within this many cells
                                          of the source (both directions); 0.5 = the source
                                          node's own cell; (0, radius[0] + 1]                  */
    int32_t subgrid;                   /* whole-grid refinement s (Section 4.5's subgrid size):
                                          0 or 1 = none; odd 3 .. 15 = the medium is refined
                                          s-fold (every fine node takes the nearest grid node's
                                          material and orientation), the fields are computed on
                                          that grid and returned at the grid's own nodes; the
                                          densities, radii and start_half_width above then count
                                          cells of the s-fold grid                             */
} ali_refine;

/* The paper's choice: densities 27, 9, 3 out to 1, 6, 13 cells; straight rays in the source
   node's own cell; no whole-grid refinement (subgrid 1).  Host only. */
void ali_default_refine(ali_refine* r);

/* Travel-time fields with nested fine grids around every source (Section 4.4) in place of
   the straight-ray box.  Per source, a sequence of grids centred on the source node, finest
   first (level l: spacing h / density[l], extending radius[l] cells and 2 fine cells around
   the source, clipped to the grid; every fine node takes the material and orientation of
   the nearest grid node).  The finest grid starts from straight rays at the source material's group
   speed inside start_half_width cells; on each level the march runs until it reaches a node
   farther than radius[l] from the source, and the nodes reached strictly earlier seed the
   next coarser grid (the nodes that coincide with them keep their times); the grid itself
   comes last.  opt->src_box_radius is not used.  Other arguments, errors and output as
   ali_solve_traveltime; ref == NULL means ali_default_refine.  Arithmetic: MIXED (the
   default) computes the fine grids in float64 (wavefront math included): with float32
   wavefront math a near tie in the score of two square stencils on a fine grid can go the
   other way and move the nodes behind it by up to 4.5e-4 on the 512 x 512 weld, beyond
   the 1e-4 bar; the grid itself is solved in the mixed arithmetic of ali_solve_traveltime.
   F64 computes everything in float64; F32 (everything in float32) is faster and outside
   the 1e-4 bar.  Scratch grows with
   the fine grids (about 23k nodes per source by default).  With ref->subgrid = s > 1 the
   grid above is the s-fold grid (spacing h / s, sources at s i, s j) and the output holds
   every s-th node of its fields; the scratch adds that grid's medium and fields (n_src
   ((nx - 1) s + 1) ((nz - 1) s + 1) travel times); a subgrid that is even, above 15, or
   makes that grid exceed 2^31 nodes is ALI_EINVAL.
   stats->ms is the host time of the call; the other counters add up every level (on the
   s-fold grid when subgrid > 1). */
ali_status ali_solve_traveltime_refined(ali_handle* h, const ali_grid* grid, const ali_material* mats,
                                        int32_t n_mats, const uint8_t* d_mat_id, const float* d_orient,
                                        const ali_node* srcs, int32_t n_src, const ali_options* opt,
                                        const ali_refine* ref, float* d_T, ali_solve_stats* stats);
ali_status ali_solve_traveltime_refined_f64(ali_handle* h, const ali_grid* grid, const ali_material* mats,
                                            int32_t n_mats, const uint8_t* d_mat_id, const double* d_orient,
                                            const ali_node* srcs, int32_t n_src, const ali_options* opt,
                                            const ali_refine* ref, double* d_T, ali_solve_stats* stats);

/* Fields of many media in one call: every source of every medium, relaxed together with
   one time threshold per field (media of different sizes progress independently).
     media[n_media]  the media (see ali_medium); 1 <= n_media
     mats[n_mats]    material table; medium m uses mats[mat_offset ..]
     d_mat_id, d_orient  per-node arrays of all media, medium m at node_offset
     srcs            sources of all media, medium m at src_offset
     d_T             output: the fields in medium order, for each medium its n_src fields of
                     [nz][nx] one after the other (float32)
   Options, arithmetic and errors as ali_solve_traveltime; stats cover the whole batch. */
ali_status ali_solve_batch(ali_handle* h, const ali_medium* media, int32_t n_media,
                           const ali_material* mats, int32_t n_mats, const uint8_t* d_mat_id,
                           const float* d_orient, const ali_node* srcs, const ali_options* opt,
                           float* d_T, ali_solve_stats* stats);

/* ali_solve_batch with the nested fine grids of ali_solve_traveltime_refined (Section 4.4)
   around every source of every medium: each level's grids, one per field, take the material
   and orientation of their own medium's nearest nodes and the materials of its range, and
   all of them relax in one call per level; the last level is the batch itself.  Media,
   layout, output and errors as ali_solve_batch; refinement, arithmetic and statistics as
   ali_solve_traveltime_refined (stats add up every level), except that ref->subgrid must
   be 0 or 1 (the s-fold medium is offered for one medium at a time; other values return
   ALI_EUNSUPPORTED).  Every field equals that of ali_solve_traveltime_refined on its own
   medium and source.  Scratch: the fine grids of all fields (about 23k nodes per field by
   default) besides that of ali_solve_batch. */
ali_status ali_solve_batch_refined(ali_handle* h, const ali_medium* media, int32_t n_media,
                                   const ali_material* mats, int32_t n_mats, const uint8_t* d_mat_id,
                                   const float* d_orient, const ali_node* srcs, const ali_options* opt,
                                   const ali_refine* ref, float* d_T, ali_solve_stats* stats);
ali_status ali_solve_batch_refined_f64(ali_handle* h, const ali_medium* media, int32_t n_media,
                                       const ali_material* mats, int32_t n_mats, const uint8_t* d_mat_id,
                                       const double* d_orient, const ali_node* srcs, const ali_options* opt,
                                       const ali_refine* ref, double* d_T, ali_solve_stats* stats);

/* Schedule autotuner: times the forward batch solve (the fields go to d_T, [field nodes]
   float32, device) under each of ALI_TUNE_CANDIDATES schedules (band_cells, inner_sweeps,
   visit_tiles, persistent) -- (1,2,4,0) (1,2,2,0) (1,2,1,0) (1,4,4,0) (2,2,4,0) (2,4,4,0)
   (1,2,4,1) -- and writes the fastest into *opt (the other fields of *opt are kept and used
   for every run).  ms_out (host, nullable) receives the time of each candidate; a
   persistent candidate whose cooperative launch the runtime refuses is left out (+inf).
   Every candidate reaches the same fields (the fixed point does not depend on the schedule);
   only the time differs.  The handle keeps the choice per size bucket (powers of two of
   the field count, the largest side and the node-fields, with the arithmetic, wave, speed
   mode and per-node stiffness): a later call for a batch of the same bucket times nothing
   and returns the kept choice and times.  Synchronises the stream. */
#define ALI_TUNE_CANDIDATES 7
ali_status ali_autotune_batch(ali_handle* h, const ali_medium* media, int32_t n_media,
                              const ali_material* mats, int32_t n_mats, const uint8_t* d_mat_id,
                              const float* d_orient, const ali_node* srcs, ali_options* opt,
                              float* d_T, double* ms_out);

/* Ray paths through finished fields (paper Section 5.1): for every source s and receiver
   r, the fastest path from r to s through field s (reciprocity), built plane by plane with
   the adaptive plane family, Fermat's principle on sampled candidates and a parabola
   through each local minimum; stops within 1.6 node spacings of the source.
     d_T            [n_src][nz][nx] fields (float32; _f64: float64), e.g. from
                    ali_solve_traveltime with the same sources
     recv[n_recv]   receiver nodes (host), inside the grid
     d_paths        [n_src][n_recv][ray_max_pts] (x, z) float pairs in grid units
     d_npts         [n_src][n_recv] number of points; negative if the ray stopped before
                    reaching the source (ray_max_pts or no usable candidate)
     d_tray         [n_src][n_recv] travel time integrated along the path [s]
   Segment times walk the nearest-node cells at the exact group speed of each cell's
   material and orientation (tabulated at 2048 angles per material). */
ali_status ali_trace_rays(ali_handle* h, const ali_grid* grid, const ali_material* mats, int32_t n_mats,
                          const uint8_t* d_mat_id, const float* d_orient, const float* d_T,
                          const ali_node* srcs, int32_t n_src, const ali_node* recv, int32_t n_recv,
                          const ali_options* opt, float* d_paths, int32_t* d_npts, float* d_tray);
ali_status ali_trace_rays_f64(ali_handle* h, const ali_grid* grid, const ali_material* mats, int32_t n_mats,
                              const uint8_t* d_mat_id, const float* d_orient, const double* d_T,
                              const ali_node* srcs, int32_t n_src, const ali_node* recv, int32_t n_recv,
                              const ali_options* opt, float* d_paths, int32_t* d_npts, float* d_tray);

/* ---- gradient with respect to the orientation ---------------------------------------- */

typedef struct {
    ali_solve_stats forward;     /* the forward solve inside the call (ms: its share)        */
    int64_t lambda_updates;      /* evaluations of the adjoint update at a node              */
    int64_t tile_visits;         /* tile passes of the adjoint relaxation                    */
    int64_t choice_mismatches;   /* nodes whose re-derived choice does not reproduce the
                                    forward value (0 unless the forward did not converge)   */
    int32_t outer_iters;         /* adjoint relaxation launches                              */
    int32_t converged;           /* 1 if the adjoint reached its fixed point                 */
    double  ms;                  /* whole call (forward + adjoint) on the stream             */
    double  relax_ms;            /* summed duration of the adjoint relaxation launches       */
} ali_adjoint_stats;

/* Gradient of a loss of the receiver travel times with respect to the orientation at
   every node (not in the paper; it differentiates the paper's update, Sections 4.2-4.4).
   The call solves the forward fields (float64 travel times, same options and result as
   ali_solve_traveltime), re-derives at every node the candidate its local update chose,
   holds those choices fixed, and runs the reverse chain rule over the resulting DAG:
       lambda(X) = dL/dT(X) + sum over nodes D whose candidate uses X of lambda(D) dU_D/dT(X)
       dL/dtheta(D) = sum over sources of lambda(D) dU_D/dtheta(D)
   plus, for the source box, lambda times the derivative of the straight-ray time with
   respect to the source node's orientation.  The result is the exact derivative of the
   discrete map wherever no stencil choice switches.  With the velocity table
   (opt->velocity = ALI_VEL_TABLE, Sections 3.2 and 4.2) the speeds are the table's
   piecewise-linear interpolants and their derivatives the slopes of the whole-degree
   intervals (the map has kinks at whole degrees as well).
     recv[n_recv]   receiver nodes (host), inside the grid
     d_dLdT         [n_src][n_recv] dL/dT at the receivers (device)
     d_T            [n_src][nz][nx] forward fields out (device, nullable)
     d_dLdtheta     [nz][nx] output (device), summed over all sources
   opt->arith must be ALI_ARITH_MIXED (float32 wavefront math in the forward, float64
   derivatives) or ALI_ARITH_F64; ALI_ARITH_F32 returns ALI_EUNSUPPORTED.  Every receiver
   must be reached by every source.  Scratch: about 62 bytes per node and source.
   Synchronises the stream. */
ali_status ali_adjoint(ali_handle* h, const ali_grid* grid, const ali_material* mats, int32_t n_mats,
                       const uint8_t* d_mat_id, const float* d_orient, const ali_node* srcs, int32_t n_src,
                       const ali_node* recv, int32_t n_recv, const float* d_dLdT, const ali_options* opt,
                       float* d_T, float* d_dLdtheta, ali_adjoint_stats* stats);
ali_status ali_adjoint_f64(ali_handle* h, const ali_grid* grid, const ali_material* mats, int32_t n_mats,
                           const uint8_t* d_mat_id, const double* d_orient, const ali_node* srcs, int32_t n_src,
                           const ali_node* recv, int32_t n_recv, const double* d_dLdT, const ali_options* opt,
                           double* d_T, double* d_dLdtheta, ali_adjoint_stats* stats);

/* ali_adjoint plus the gradient with respect to the stiffness of every node (not in the
   paper; it differentiates the same updates, Sections 3.2 and 4.2-4.4).  The parameters are
   the density-normalised stiffnesses A = C / rho of each node's material, in the order
   A11, A13, A33, A55 [m^2/s^2] (the in-plane qP speeds depend on these only), each node
   treated as a parameter of its own.  A stencil estimate depends on its node's A through the
   phase speed at the wavefront normal; a straight-ray time (fallback or source box) through
   the exact group speed at a fixed group angle, whose derivative is (V / v) dv/dA at the
   phase angle that carries that group angle (envelope theorem); source-box terms go to the
   source node.
     d_dLdA         [nz][nx][4] output (device), summed over all sources; NULL is an error
   Gradients w.r.t. C and rho follow by the chain rule: dL/dC = dL/dA / rho and
   dL/drho = -sum_k A_k dL/dA_k / rho.  The velocity table returns ALI_EUNSUPPORTED.  Every
   other argument, the arithmetic, errors and synchronisation as ali_adjoint.  Scratch: 40
   more bytes per node and source. */
ali_status ali_adjoint_stiffness(ali_handle* h, const ali_grid* grid, const ali_material* mats, int32_t n_mats,
                                 const uint8_t* d_mat_id, const float* d_orient, const ali_node* srcs,
                                 int32_t n_src, const ali_node* recv, int32_t n_recv, const float* d_dLdT,
                                 const ali_options* opt, float* d_T, float* d_dLdtheta, float* d_dLdA,
                                 ali_adjoint_stats* stats);
ali_status ali_adjoint_stiffness_f64(ali_handle* h, const ali_grid* grid, const ali_material* mats,
                                     int32_t n_mats, const uint8_t* d_mat_id, const double* d_orient,
                                     const ali_node* srcs, int32_t n_src, const ali_node* recv, int32_t n_recv,
                                     const double* d_dLdT, const ali_options* opt, double* d_T,
                                     double* d_dLdtheta, double* d_dLdA, ali_adjoint_stats* stats);

/* Forward + adjoint for the travel-time misfit L = 1/2 sum over (s, r) of
   (T_s(r) - obs[s][r])^2 in one call (the tomography step).
     d_obs          [n_src][n_recv] observed times (device)
     d_T            [n_src][nz][nx] forward fields out (device, nullable)
     d_Trec         [n_src][n_recv] modelled times at the receivers (device, nullable)
     d_loss         one float64 on the device: L (nullable)
     d_dLdtheta     [nz][nx] dL/dtheta (device)
   Arithmetic, errors and synchronisation as ali_adjoint. */
ali_status ali_misfit_gradient(ali_handle* h, const ali_grid* grid, const ali_material* mats, int32_t n_mats,
                               const uint8_t* d_mat_id, const float* d_orient, const ali_node* srcs,
                               int32_t n_src, const ali_node* recv, int32_t n_recv, const float* d_obs,
                               const ali_options* opt, float* d_T, float* d_Trec, double* d_loss,
                               float* d_dLdtheta, ali_adjoint_stats* stats);
ali_status ali_misfit_gradient_f64(ali_handle* h, const ali_grid* grid, const ali_material* mats,
                                   int32_t n_mats, const uint8_t* d_mat_id, const double* d_orient,
                                   const ali_node* srcs, int32_t n_src, const ali_node* recv, int32_t n_recv,
                                   const double* d_obs, const ali_options* opt, double* d_T, double* d_Trec,
                                   double* d_loss, double* d_dLdtheta, ali_adjoint_stats* stats);

/* ali_misfit_gradient of the forward on the medium refined s-fold (Section 4.5's subgrid
   size s; the forward of ali_solve_traveltime_refined with ref->subgrid = s and no nested
   source grids): the ((nx - 1) s + 1) x ((nz - 1) s + 1) grid of spacing h / s whose nodes
   take the material and orientation of the nearest node, the sources and receivers on its
   nodes (s i, s j) and the straight-ray source box of opt->src_box_radius fine nodes.  Each
   node's orientation reaches the fine nodes nearest to it, so d_dLdtheta [nz][nx] is the
   s-fold grid's gradient summed over those nodes (the chain rule through the refinement).
     subgrid        1 (ali_misfit_gradient itself) or odd in [3, 15]; else ALI_EINVAL
     d_T            [n_src][nz][nx] the s-fold fields at the nodes (device, nullable)
   Every other argument as ali_misfit_gradient; opt->d_node_A returns ALI_EUNSUPPORTED.
   Scratch: that of ali_misfit_gradient on the s-fold grid plus 9 bytes per fine node
   (float64 entry: 17) and, with d_T, one travel time per fine node and source.
   Synchronises the stream. */
ali_status ali_misfit_gradient_subgrid(ali_handle* h, const ali_grid* grid, const ali_material* mats,
                                       int32_t n_mats, const uint8_t* d_mat_id, const float* d_orient,
                                       const ali_node* srcs, int32_t n_src, const ali_node* recv, int32_t n_recv,
                                       const float* d_obs, const ali_options* opt, int32_t subgrid, float* d_T,
                                       float* d_Trec, double* d_loss, float* d_dLdtheta, ali_adjoint_stats* stats);
ali_status ali_misfit_gradient_subgrid_f64(ali_handle* h, const ali_grid* grid, const ali_material* mats,
                                           int32_t n_mats, const uint8_t* d_mat_id, const double* d_orient,
                                           const ali_node* srcs, int32_t n_src, const ali_node* recv,
                                           int32_t n_recv, const double* d_obs, const ali_options* opt,
                                           int32_t subgrid, double* d_T, double* d_Trec, double* d_loss,
                                           double* d_dLdtheta, ali_adjoint_stats* stats);

/* ali_misfit_gradient plus dL/dA [nz][nx][4] of every node's stiffness (as
   ali_adjoint_stiffness; NULL is an error). */
ali_status ali_misfit_gradient_stiffness(ali_handle* h, const ali_grid* grid, const ali_material* mats,
                                         int32_t n_mats, const uint8_t* d_mat_id, const float* d_orient,
                                         const ali_node* srcs, int32_t n_src, const ali_node* recv, int32_t n_recv,
                                         const float* d_obs, const ali_options* opt, float* d_T, float* d_Trec,
                                         double* d_loss, float* d_dLdtheta, float* d_dLdA, ali_adjoint_stats* stats);
ali_status ali_misfit_gradient_stiffness_f64(ali_handle* h, const ali_grid* grid, const ali_material* mats,
                                             int32_t n_mats, const uint8_t* d_mat_id, const double* d_orient,
                                             const ali_node* srcs, int32_t n_src, const ali_node* recv,
                                             int32_t n_recv, const double* d_obs, const ali_options* opt,
                                             double* d_T, double* d_Trec, double* d_loss, double* d_dLdtheta,
                                             double* d_dLdA, ali_adjoint_stats* stats);

/* Forward + adjoint of the travel-time misfit for many media in one call (the batched
   tomography step): for each medium m, L_m = 1/2 sum over its sources s and receivers r of
   (T_s(r) - obs)^2.
     recv            receivers of all media, medium m at rec_offset (n_rec of them)
     d_obs           observed times: for each field (medium order, then source order) its
                     medium's n_rec values
     d_Trec          modelled times, same layout (device, nullable)
     d_loss          [n_media] float64 misfits (device, nullable)
     d_dLdtheta      dL_m/dtheta per node, laid out as d_orient (device)
   Arithmetic, errors and synchronisation as ali_misfit_gradient. */
ali_status ali_misfit_gradient_batch(ali_handle* h, const ali_medium* media, int32_t n_media,
                                     const ali_material* mats, int32_t n_mats, const uint8_t* d_mat_id,
                                     const float* d_orient, const ali_node* srcs, const ali_node* recv,
                                     const float* d_obs, const ali_options* opt, float* d_Trec,
                                     double* d_loss, float* d_dLdtheta, ali_adjoint_stats* stats);
/* The same plus dL_m/dA of every node's stiffness, 4 values per node laid out as d_orient
   (as ali_adjoint_stiffness; NULL is an error). */
ali_status ali_misfit_gradient_batch_stiffness(ali_handle* h, const ali_medium* media, int32_t n_media,
                                               const ali_material* mats, int32_t n_mats, const uint8_t* d_mat_id,
                                               const float* d_orient, const ali_node* srcs, const ali_node* recv,
                                               const float* d_obs, const ali_options* opt, float* d_Trec,
                                               double* d_loss, float* d_dLdtheta, float* d_dLdA,
                                               ali_adjoint_stats* stats);

/* Orientation from an ncz x ncx grid of control values spanning the grid corner to corner
   (node k sits at control coordinate k (nc-1)/(n-1); linear in each direction), and its
   transpose, which maps dL/dtheta [nz][nx] to dL/dcontrol [ncz][ncx].  Needs nz, nx, ncz,
   ncx >= 2 and ncz <= nz, ncx <= nx.  Device arrays; asynchronous. */
ali_status ali_bilinear(ali_handle* h, int32_t nz, int32_t nx, int32_t ncz, int32_t ncx,
                        const float* d_ctrl, float* d_orient);
ali_status ali_bilinear_transpose(ali_handle* h, int32_t nz, int32_t nx, int32_t ncz, int32_t ncx,
                                  const float* d_dLdtheta, float* d_dLdctrl);
ali_status ali_bilinear_f64(ali_handle* h, int32_t nz, int32_t nx, int32_t ncz, int32_t ncx,
                            const double* d_ctrl, double* d_orient);
ali_status ali_bilinear_transpose_f64(ali_handle* h, int32_t nz, int32_t nx, int32_t ncz, int32_t ncx,
                                      const double* d_dLdtheta, double* d_dLdctrl);

#ifdef __cplusplus
}
#endif
#endif
