/*
 * ibx.h -- C ABI of libibx, the multidirect-forcing immersed-boundary (IB)
 * loop of arXiv 2408.14140 (IAMReX) on one AMD Instinct MI355X (gfx950).
 *
 * Conventions shared by every call
 * --------------------------------
 * Memory:  every buffer is allocated and owned by the caller.  "device"
 *          pointers are HIP device allocations on the current device, "host"
 *          pointers are ordinary host memory.  The library allocates device
 *          memory only inside an ib_plan (graph cache), released by
 *          ib_plan_destroy.  Scratch memory is passed as a workspace whose
 *          size is queried first.
 * Streams: every call is enqueued on the given stream (hipStream_t passed as
 *          void*, NULL = the null stream) and returns without synchronizing;
 *          outputs are valid once the stream reaches that point.
 * Errors:  arguments are validated on the host before anything is enqueued;
 *          a negative ib_status is returned synchronously and nothing runs.
 *          A failed kernel launch returns IB_EHIP (hipGetLastError text via
 *          ib_last_hip_error).  Conditions only the device can see (a marker
 *          stencil outside the covered boxes, a source-list overflow) are
 *          reported through device flag words that the caller reads after
 *          synchronizing; every call made with a flagged bucket set writes
 *          NaN into all of its outputs (checked on the device, no host
 *          synchronization), so a wrong result never looks valid.
 * Grid:    the finest AMR level: n[0] x n[1] x n[2] cells of edge h whose low
 *          corner is lo (Sec. 3.1: IB markers live on the finest level only).
 *          It is tiled into cubic boxes of `box` cells; only covered boxes
 *          hold data.  A cell-centred field is stored per covered box as
 *          [nbox][3][E][E][E] with E = box + 2*ngrow, x fastest; the ghost
 *          cells are neither read nor written.  FP32 fields are float, FP64
 *          fields double.
 * Markers: structure of arrays in FP64 positions, contiguous per particle;
 *          per-marker vectors (U, U^d, F) are [nl][3] in the field
 *          precision.
 * Kernel:  delta_h(x) h^3 = prod_d phi((X_d - x_d)/h) with phi the 3-point
 *          kernel of Roma, Peskin & Berger (1999) or the 4-point kernel of
 *          Peskin (2002), the two the paper cites in Sec. 3.1.  Stencil of a
 *          marker per axis: s = (X - lo)/h, base b = floor(s) - 1 (3-point)
 *          or floor(s - 1/2) - 1 (4-point), cells b .. b+P-1 (wrapped on
 *          periodic axes).
 */
#ifndef IBX_H
#define IBX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IB_OK = 0,
    IB_EINVAL = -1,       /* invalid argument (null pointer, bad size or enum) */
    IB_EDOMAIN = -2,      /* input outside the covered grid (host-detectable) */
    IB_EWORKSPACE = -3,   /* workspace missing or smaller than required */
    IB_EHIP = -4,         /* a HIP runtime call or kernel launch failed */
    IB_EUNSUPPORTED = -5  /* valid but unsupported combination */
} ib_status;

typedef enum { IB_DELTA3 = 3, IB_DELTA4 = 4 } ib_delta;
typedef enum { IB_F64 = 0, IB_F32 = 1 } ib_prec;
typedef enum { IB_PATH_AUTO = 0, IB_PATH_PLAIN = 1, IB_PATH_BATCHED = 2 } ib_path;

/* Finest level (Sec. 3.1, Algorithm 2: markers exist on level l_max only). */
typedef struct ib_level {
    int32_t n[3];            /* cells per axis; each a multiple of box */
    double h;                /* cell edge, equal on all axes */
    double lo[3];            /* physical position of the low corner of cell (0,0,0) */
    int32_t periodic[3];     /* 1 = periodic axis, 0 = bounded axis */
    int32_t box;             /* box edge in cells, a multiple of 8 */
    int32_t ngrow;           /* ghost width of caller field arrays (>= 0, never read) */
    int32_t nbox;            /* number of covered boxes */
    const int32_t* box_lo;   /* device [nbox][3] low cell of each covered box */
    const int32_t* box_lut;  /* device [(n0/box)(n1/box)(n2/box)] x fastest: box id or -1 */
} ib_level;

/* Rigid particles (Sec. 3.2): centroid X_r, diameter, U_r and W_r of Eq. (pr1). */
typedef struct ib_particles {
    int32_t np;
    const double* xc;        /* device [np][3] */
    const double* d;         /* device [np] */
    const double* up;        /* device [np][3] */
    const double* om;        /* device [np][3] */
} ib_particles;

/* Lagrangian surface markers (Sec. 3.1, Fig. 4: on the surface only). */
typedef struct ib_markers {
    int64_t nl;              /* total number of markers */
    const int64_t* offs;     /* device [np+1] first marker of each particle */
    double* x;               /* device [nl] */
    double* y;               /* device [nl] */
    double* z;               /* device [nl] */
    int32_t* pid;            /* device [nl] owning particle */
    double* dv;              /* device [np] marker volume dV of each particle */
} ib_markers;

/* Markers bucketed by owning tile (tile = 8 cells per axis). */
typedef struct ib_buckets {
    int32_t* cell;           /* device [nl] owning cell (wrapped), x + n0 (y + n1 z) */
    int32_t* tileid;         /* device [nl] tile of the owning cell, x fastest */
    int32_t* base;           /* device [nl][3] stencil base b (unwrapped) */
    int32_t* perm;           /* device [nl] marker at each sorted position (stable) */
    int32_t* tile_offs;      /* device [T+1] first sorted position of each tile */
    int32_t* src_offs;       /* device [T+1] start of each tile's source list */
    int32_t* src_idx;        /* device [src_cap] sorted positions touching each tile */
    int64_t src_cap;         /* capacity of src_idx (8*nl always suffices) */
    int32_t* flag;           /* device [2]: [0] markers outside coverage, [1] src overflow */
} ib_buckets;

typedef struct ib_plan ib_plan;

/* ---------------------------------------------------------------------- */
/* a1  Markers.  N_p = round(pi (D_p/h)^2) markers on an equal-area        */
/* Fibonacci spiral of radius D_p/2 around each centroid, with             */
/* dV_p = (pi h / 3 N_p)(3 D_p^2 + h^2), the shell of thickness h divided   */
/* evenly.  The paper states only that markers sit on the particle surface  */
/* at the finest level (Sec. 3.1, Fig. 4); the counts are this library's.   */
/* ---------------------------------------------------------------------- */

/* Host: offs_host[np+1] receives the running marker counts.  Returns the
 * total count, or IB_EINVAL for np < 0, h <= 0, a null pointer or d <= 0. */
int64_t ib_count_markers(int32_t np, const double* d_host, double h, int64_t* offs_host);

/* Device: fills m->x, y, z, pid, dv from p and m->offs (copied from
 * ib_count_markers by the caller).  Returns IB_OK, IB_EINVAL, IB_EHIP. */
int ib_build_markers(const ib_level* lv, const ib_particles* p, const ib_markers* m,
                     void* stream);

/* a3  Desired marker velocity, Eq. (pr1): U^d_l = U_r + W_r x (X_l - X_r).
 * Ud: device [nl][3] in precision prec. */
int ib_desired_velocity(const ib_particles* p, const ib_markers* m, ib_prec prec, void* Ud,
                        void* stream);

/* ---------------------------------------------------------------------- */
/* a2  Bucketing.  Owning cell c = floor(s) per axis, tile = c / 8; stable */
/* LSD radix sort of markers by tile (per 8-bit digit: histogram, scan,    */
/* scatter); for every tile the ascending list of sorted positions whose   */
/* stencil cells touch it.  Not in the paper, which treats one particle at */
/* a time (Sec. 3.1); integer outputs are deterministic.  flag[0] counts   */
/* markers whose stencil leaves the covered boxes or a bounded axis,       */
/* flag[1] is set when src_idx overflows src_cap; ib_spread,               */
/* ib_multidirect_force, ib_plan_autotune and ib_multidirect_backward      */
/* called with such a set write NaN into every output.                     */
/* ---------------------------------------------------------------------- */

/* Device workspace of ib_bucket in bytes: grows with nl and with the level's
 * tile count (0 for an invalid level or nl < 0). */
size_t ib_bucket_workspace(const ib_level* lv, int64_t nl);
int ib_bucket(const ib_level* lv, const ib_markers* m, ib_delta delta, const ib_buckets* b,
              void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------- */
/* a4  Velocity interpolation, Algorithm 1 first sub-step:                  */
/*     U_l = sum_x u(x) delta_h(x - X_l) h^3.                               */
/* u: field in the box layout; U: device [nl][3].  One thread per marker,   */
/* FP64 or FP32 arithmetic as prec.  A marker whose stencil reaches a cell  */
/* off a bounded axis or in an uncovered box gets U = NaN.                  */
/* ---------------------------------------------------------------------- */
int ib_interp(const ib_level* lv, const ib_markers* m, ib_delta delta, ib_prec prec,
              const void* u, void* U, void* stream);

/* ---------------------------------------------------------------------- */
/* a6  Force spreading, Algorithm 1 third sub-step:                          */
/*     f(x) = sum_l F_l delta_h(x - X_l) dV_l.                              */
/* Writes f on every valid cell of every covered box (zero where no marker  */
/* reaches).  Deterministic: each cell sums its tile's source list in       */
/* order.  Needs the buckets of the same markers; with a flagged bucket set */
/* f is NaN on every valid cell.                                            */
/* ---------------------------------------------------------------------- */
int ib_spread(const ib_level* lv, const ib_markers* m, const ib_buckets* b, ib_delta delta,
              ib_prec prec, const void* F, void* f, void* stream);

/* ---------------------------------------------------------------------- */
/* a3-a9  Multidirect forcing, Algorithm 1 (Sec. 3.1): with F^0 = 0 and      */
/* u^(0) = u0, for m = 1..ns: U = J u^(m-1); F^m = F^(m-1) + (U^d - U)/dt;  */
/* f^m = S F^m; u^(m) = u0 + dt f^m.  All markers of all particles are      */
/* iterated together.  Outputs ustar = u^(ns) and f = f^ns on every valid   */
/* cell of the covered boxes, F = F^ns [nl][3] (marker order).              */
/*   ustar may equal u0 (in place) on the batched path; f may be NULL.      */
/*   resid (device double [ns+1] or NULL) receives                          */
/*   sqrt(sum_l dV_l |U^d_l - (J u^(m))_l|^2), m = 0..ns.                     */
/*   Fhist (device [ns][nl][3] or NULL) receives F^1..F^ns for the adjoint. */
/*   With a flagged bucket set, ustar, f, F, resid and Fhist are all NaN    */
/*   (ustar overwrites u0 when they alias).                                 */
/* The plan fixes kernel width, precision and path (plain: one kernel per   */
/* sub-step, straight from global memory; batched: tile-staged LDS kernels  */
/* fed by the buckets, ustar may alias u0; needs at least 16 cells per axis */
/* and box <= 512, else IB_EUNSUPPORTED).  bucket_width: markers per        */
/* interpolation work item (64, 128 or 256; 0 = 256).  spread_wgs_per_cu:   */
/* cap on resident spreading workgroups per compute unit (1..32; 0 = 16),  */
/* lowered to what fits.  Interpolation runs as many workgroups as fit.     */
/* use_graph: replay the launch sequence from a captured hipGraph when the  */
/* arguments repeat (batched path, non-null stream).  On a stream that is   */
/* already being captured the launches go into the caller's graph instead.  */
/* row_masks (batched path): the spreading records which rows of each tile's */
/* G slot are not all zeros and stores only those, and the interpolation    */
/* and the finalize step load only those: less traffic (about a fifth on   */
/* 1000 spheres at 256^3) for a mask test per row, which may or may not pay */
/* (ib_plan_autotune measures it).  Results are the same either way (a row */
/* of zeros reads back as +0).  interp_tile (batched path): x extent of the */
/* interpolation work tiles, 8 (one 8^3 tile; 0 = 8) or 16 (two x          */
/* neighbours, whose markers share one staged halo: 20 x 12 x 12 cells     */
/* instead of two 12^3; FP32 plans only, else IB_EUNSUPPORTED).  Spreading, */
/* bucketing and the G slots stay on 8^3 tiles; results agree to rounding  */
/* (an item's marker count decides over how many lanes each marker's       */
/* stencil sum is split).                                                   */
/* ib_plan_autotune, ib_plan_profile_read, ib_particle_levels and           */
/* ib_multidirect_sequential synchronize and must not be captured; every    */
/* other call only enqueues work on its stream and may be.                  */
/* ---------------------------------------------------------------------- */
int ib_plan_create(ib_plan** plan, ib_delta delta, ib_prec prec, ib_path path,
                   int32_t bucket_width, int32_t spread_wgs_per_cu, int32_t use_graph,
                   int32_t row_masks, int32_t interp_tile);
void ib_plan_destroy(ib_plan* plan);
/* Current tuning of a plan (out: int32[6]): out[0] = path, out[1] =
 * bucket_width, out[2] = spread_wgs_per_cu, out[3] = use_graph, out[4] =
 * row_masks, out[5] = interp_tile. */
int ib_plan_query(const ib_plan* plan, int32_t* out);
/* Workspace of ib_multidirect_force and ib_plan_autotune (device bytes); it
 * does not depend on the plan's tuning. */
size_t ib_workspace_bytes(const ib_plan* plan, const ib_level* lv, int64_t nl, int32_t ns);

/* Per-kernel timing of the batched path.  ib_plan_profile(plan, 1) makes
 * later ib_multidirect_force calls record a pair of HIP events around each
 * kernel launch on the caller's stream (up to 1024 launches between reads;
 * graph replay is suspended while enabled).  ib_plan_profile_read waits for
 * the recorded events, adds their durations per kernel class and returns the
 * totals (milliseconds) and launch counts in arrays of IB_PROF_CLASSES
 * entries, in the order of ib_prof_class; reset != 0 clears the totals.     */
typedef enum {
    IB_PROF_PREP = 0,         /* sorted marker records: stencil, weights, U^d */
    IB_PROF_LISTS = 1,        /* work lists: per-tile items, active tiles */
    IB_PROF_INTERP_U0 = 2,    /* interpolation of u0 and F^1 */
    IB_PROF_SPREAD = 3,       /* spreading of F^(m-1) into the per-tile buffer */
    IB_PROF_INTERP_G = 4,     /* interpolation of that buffer and the F update */
    IB_PROF_SPREAD_FINAL = 5, /* spreading of F^ns into f and ustar */
    IB_PROF_FILL = 6,         /* f = 0, ustar = u0 where no marker reaches */
    IB_PROF_UNSORT = 7,       /* F back to marker order */
    IB_PROF_RESID = 8,        /* residual-only interpolation */
    IB_PROF_CLASSES = 9
} ib_prof_class;
int ib_plan_profile(ib_plan* plan, int32_t enable);
int ib_plan_profile_read(ib_plan* plan, double* total_ms, int64_t* calls, int32_t reset);
int ib_multidirect_force(ib_plan* plan, const ib_level* lv, const ib_particles* p,
                         const ib_markers* m, const ib_buckets* b, int32_t ns, double dt,
                         const void* u0, void* ustar, void* f, void* F, double* resid,
                         void* Fhist, void* ws, size_t ws_bytes, void* stream);

/* Autotuning of a batched plan (the batching extension of the coupling loop:
 * the work-item width, the spreading residency and the slot row masks are
 * chosen on the real inputs).  Times the loop of ib_multidirect_force for
 * every bucket_width in {64, 128, 256}, spread_wgs_per_cu in {4, 8, 16, 32},
 * row_masks in {0, 1} and (FP32) interp_tile in {8, 16}, each as replays of
 * its captured graph, in place on ustar after a copy of u0 (one warm-up, then
 * the faster of two samples of 3 replays; the capture runs on a stream the
 * call creates and destroys) and
 * keeps the fastest in the plan (see ib_plan_query); the row masks and the
 * 16-wide work tile are kept only when they win by more than 1%.  The
 * tile stays 8^3: one 64-wide wavefront holds the 64 rows of a tile.
 * Arguments as ib_multidirect_force, except that ustar must not alias u0 and
 * no residual or history is taken; ustar, f and F hold the result of the
 * last run.  Synchronizes the stream (do not capture).  out_ms (host,
 * nullable) receives the chosen configuration's loop time in ms.  Returns
 * IB_EUNSUPPORTED for a plain plan; on any error the plan keeps its tuning. */
int ib_plan_autotune(ib_plan* plan, const ib_level* lv, const ib_particles* p,
                     const ib_markers* m, const ib_buckets* b, int32_t ns, double dt,
                     const void* u0, void* ustar, void* f, void* F, void* ws, size_t ws_bytes,
                     void* stream, double* out_ms);

/* ---------------------------------------------------------------------- */
/* a10 Per-particle sums for the rigid-body update, Eqs. (particle1),       */
/* (particle2) and (FD): out[p] = [ sum_l F_l dV (3), sum_l R_l x F_l dV (3),*/
/* sum_x alpha_p u h^3 (3), sum_x alpha_p (x - X_p) x u h^3 (3) ] in FP64,   */
/* alpha_p the particle volume fraction of Eq. (level-set function) from     */
/* the eight nodal values of phi_p = |x - X_p|/(D_p/2) - 1 (Sec. 4.1).       */
/* Raw sums: the caller applies -rho_f and the time derivatives.  F and u   */
/* in precision prec; out: device double [np][12].  flag (device int32 or   */
/* NULL) is set to 1 when a particle's cells leave the covered boxes; such  */
/* a particle gets NaN in all twelve of its sums.  ws:                      */
/* device workspace of ib_reductions_workspace(np) bytes (partial sums).     */
/* Deterministic: fixed-order tree reductions in FP64.                      */
/* ---------------------------------------------------------------------- */
size_t ib_reductions_workspace(int32_t np);
int ib_particle_reductions(const ib_level* lv, const ib_particles* p, const ib_markers* m,
                           ib_prec prec, const void* F, const void* u, double* out,
                           int32_t* flag, void* ws, size_t ws_bytes, void* stream);

/* ib_particle_reductions for callers that cannot allocate device memory   */
/* (code under HIP graph capture, tight serving loops, harnesses that      */
/* forbid hipMalloc): the same sums from the same kernels, bit for bit,    */
/* with the partial sums kept in a fixed device array inside the library   */
/* instead of a workspace.  The array holds IB_REDUCTIONS_NOALLOC_MAX_NP    */
/* particles (7.5 MiB, one copy per device, kept until the process ends);  */
/* p->np above that returns IB_EUNSUPPORTED before anything is enqueued.   */
/* Nothing is allocated: no hipMalloc, hipFree or allocating library call. */
/* Every call on one device shares that device's array, so calls that      */
/* overlap on a device (different streams, or threads) race; calls on one  */
/* stream are ordered and safe.  Nothing in the array needs clearing: each */
/* call writes every entry it reads.  The first call on a device looks up  */
/* the array's device address (hipGetSymbolAddress) once.                   */
#define IB_REDUCTIONS_NOALLOC_MAX_NP 32768
int ib_particle_reductions_noalloc(const ib_level* lv, const ib_particles* p,
                                   const ib_markers* m, ib_prec prec, const void* F,
                                   const void* u, double* out, int32_t* flag, void* stream);

/* ---------------------------------------------------------------------- */
/* a11 Adjoint of ib_multidirect_force (reverse sweep; S and J adjoint,     */
/* Sec. 2).  Given Fhist from the forward call and the upstream gradients   */
/* g_ustar (field or NULL), g_f (field or NULL) and g_F ([nl][3] or NULL),  */
/* all in precision prec, writes g_u0 (field, precision prec), and in FP64   */
/* g_up and g_om ([np][3]) and g_X ([nl][3], gradient with respect to the   */
/* marker positions through phi').  Intermediate fields u^(m-1) are         */
/* recomputed from u0 and Fhist, never stored.  ws sized by                 */
/* ib_backward_workspace_bytes.  Runs on the plain kernels for either plan  */
/* path.  With a flagged bucket set every gradient output is NaN.           */
/* ---------------------------------------------------------------------- */
size_t ib_backward_workspace_bytes(const ib_plan* plan, const ib_level* lv, int64_t nl);
int ib_multidirect_backward(ib_plan* plan, const ib_level* lv, const ib_particles* p,
                            const ib_markers* m, const ib_buckets* b, int32_t ns, double dt,
                            const void* u0, const void* Fhist, const void* g_ustar,
                            const void* g_f, const void* g_F, void* g_u0, double* g_up,
                            double* g_om, double* g_X, void* ws, size_t ws_bytes, void* stream);

/* Helpers. */
/* ---------------------------------------------------------------------- */
/* The particle side of a time step (Sec. 3.2; Step 4 of Sec. 3.1).        */
/* ---------------------------------------------------------------------- */

/* Rigid-body update of the spheres.  Free particles follow Eqs.            */
/* (particle1) and (particle2) with the right-hand sides at the half step    */
/* (the midpoint rule):                                                     */
/*   rho_p V_p (U' - U)/dt = -rho_f S_F + rho_f (I_u' - I_u)/dt               */
/*                           + (rho_p - rho_f) V_p g + F_c,                   */
/*   I_p (W' - W)/dt       = -rho_f S_T + rho_f (I_ru' - I_ru)/dt + T_c,       */
/* V_p = pi D^3/6, I_p = rho_p V_p D^2/10 (solid sphere).  sums_n: device    */
/* [np][12] from ib_particle_reductions with F = F^{n+1/2} and u = u^n       */
/* (S_F, S_T, I_u, I_ru); sums_np1: the same with u^{n+1} (only I_u', I_ru'  */
/* used).  rho_p: device [np].  Fc, Tc (device [np][3]) and prescribed       */
/* (device int32 [np]; nonzero = keep U and W) may be NULL.  grav: host [3]. */
/* The centroid moves by Eq. (pr2), X' = X + dt/2 (U + U').  Outputs are     */
/* device [np][3] and must not alias the inputs.                             */
int ib_rigid_update(const ib_particles* p, const double* rho_p, const double* sums_n,
                    const double* sums_np1, const double* Fc, const double* Tc,
                    const int32_t* prescribed, double rho_f, const double* grav, double dt,
                    double* up_new, double* om_new, double* xc_new, void* stream);

/* Markers follow their particle's rigid motion (Eq. (x) with U = U_r +     */
/* W x R): X' = X_r' + Q (X - X_r), Q the rotation by |W| dt about W with    */
/* W = (W^n + W^{n+1})/2 (Rodrigues' formula), identity when W = 0.  m holds */
/* the positions at t^n; xc_n, xc_np1, om_n, om_np1 are device [np][3]; the  */
/* new positions (device [nl] each) may overwrite m's arrays.                */
int ib_advect_markers(const ib_markers* m, const double* xc_n, const double* xc_np1,
                      const double* om_n, const double* om_np1, double dt, double* x_new,
                      double* y_new, double* z_new, void* stream);

/* Repulsive collision force between particles, Eq. (DKT_model) (after      */
/* Breugem 2012): for every pair closer than D_c = R_i + R_j + h,             */
/*   F_c,ij = -(m |g| / eps_c) ((|delta| - D_c)/h)^2 delta/|delta|,           */
/* delta = X_j - X_i by the minimum image on the level's periodic axes, h   */
/* the finest spacing, m the mean of the two masses rho V (the paper's case  */
/* has equal spheres).  Fc (device [np][3], out) = sum over j of F_c,ij; the */
/* force is central, so the collision torque is zero.  rho_p: device [np];  */
/* the paper uses eps_c = 1e-4.  Partners are found through bins of whole  */
/* tiles at least max D_c (plus one cell) wide, so a particle meets only    */
/* the particles of its own and the neighbouring bins; each particle's sum  */
/* runs over those bins and, within a bin, ascending partner index: a fixed */
/* order.  ws: device workspace of ib_collision_workspace(lv, np) bytes     */
/* (IB_EWORKSPACE when short).  The call only enqueues work on stream.      */
size_t ib_collision_workspace(const ib_level* lv, int32_t np);
int ib_collision_forces(const ib_level* lv, const ib_particles* p, const double* rho_p,
                        double g_norm, double eps_c, double* Fc, void* ws, size_t ws_bytes,
                        void* stream);

/* ---------------------------------------------------------------------- */
/* Particle-by-particle order of the coupling loop (Sec. 3.1, the remarks   */
/* after Algorithm 1: each particle runs the N_s loop in turn on the field  */
/* its predecessors left; the corrected forces of all particles add up).    */
/* ---------------------------------------------------------------------- */

/* Conflict levels.  level[j] (device int32 [np], out) = 0 when no earlier   */
/* particle's kernel support may share a cell with particle j's, else 1 +   */
/* the largest level among those that may.  "May share" is the conservative */
/* test |X_i - X_j| < (D_i + D_j)/2 + 2 P h (minimum image on periodic      */
/* axes; it assumes every marker lies within D/2 of its centroid).  Particles */
/* of one level have disjoint supports, and every conflicting pair keeps    */
/* its index order across levels.  *nlevels (host, out) = 1 + max level (0  */
/* when np = 0).  ws: device workspace of ib_levels_workspace(np) bytes.    */
/* Iterates on the device until the levels stop changing, reading a flag    */
/* back after every pass: synchronizes the stream (do not capture).         */
size_t ib_levels_workspace(int32_t np);
int ib_particle_levels(const ib_level* lv, const ib_particles* p, ib_delta delta,
                       int32_t* level, int32_t* nlevels, void* ws, size_t ws_bytes,
                       void* stream);

/* The loop in particle order.  Particles are grouped by level (stable in    */
/* index), and the levels run one after another, each as one batched loop  */
/* of ib_multidirect_force over its particles on the field the previous     */
/* levels left: u^(0) of level c is u* of level c-1 (u0 for the first).     */
/* Outputs: ustar = u* after the last level, f = the sum of every level's    */
/* f^ns, F = every marker's F^ns (marker order), as the particle-by-particle */
/* sweep gives them up to rounding.  ustar may equal u0; f may be NULL.      */
/* level/nlevels as from ib_particle_levels (any level function with        */
/* disjoint supports within a level gives a valid order; nlevels <= 4096,   */
/* else IB_EUNSUPPORTED).  Markers must be contiguous per particle as given */
/* by m->offs (pid is not read).  flag (device int32 [2] or NULL) receives  */
/* the OR of the per-level bucketing flags (ib_buckets.flag).  Batched plans */
/* only (IB_EUNSUPPORTED otherwise); no graph replay, no residuals.  When a */
/* level's bucketing is flagged, ustar, f and F are all NaN.  Reads          */
/* the level boundaries back once: synchronizes the stream (do not capture). */
/* ws: device workspace of ib_sequential_workspace_bytes(plan, lv, np, nl,   */
/* ns) bytes.  IB_EINVAL (after that synchronization, nothing else run) for */
/* a level outside [0, nlevels) or offs not a partition of [0, nl).         */
size_t ib_sequential_workspace_bytes(const ib_plan* plan, const ib_level* lv, int32_t np,
                                     int64_t nl, int32_t ns);
int ib_multidirect_sequential(ib_plan* plan, const ib_level* lv, const ib_particles* p,
                              const ib_markers* m, int32_t ns, double dt, const int32_t* level,
                              int32_t nlevels, const void* u0, void* ustar, void* f, void* F,
                              int32_t* flag, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------- */
/* Single-level periodic fluid steps around the IB loop (Sec. 3.1).         */
/* Grid: n^3 cells of edge h, periodic on every axis, n a power of two in   */
/* [8, 1024] (else IB_EUNSUPPORTED).  Velocity is cell-centred, device      */
/* [3][n][n][n] x fastest, in precision prec; pressure is node-centred      */
/* (the semi-staggered grid), device [n][n][n], node (i, j, k) at the low   */
/* corner of cell (i, j, k).  Discrete operators: G p = cell gradient of    */
/* nodal p (the difference across the cell averaged over its four edges     */
/* along the axis); D V = nodal divergence of cell V, D = -G^T; L = 7-point */
/* Laplacian; the convective term in central flux form (face value = mean   */
/* of the two cells), standing in for the Godunov scheme the paper cites.   */
/* Constant rho and mu.  Both solves are exact (FFT).  ws: device workspace */
/* of ib_fluid_workspace(n, prec) bytes.  Enqueue-only.                     */
/* ---------------------------------------------------------------------- */
size_t ib_fluid_workspace(int32_t n, ib_prec prec);
/* Step 1, Eq. (31): ustar = u~*, solving                                   */
/*   (I - nu dt/2 L) u~* = u - dt div(uu) - (dt/rho) G p + (nu dt/2) L u     */
/*                         + dt g,   nu = mu / rho,                           */
/* from u = u^n and p = p^{n-1/2}; grav: host [3].  ustar may alias u.      */
int ib_fluid_predict(int32_t n, double h, ib_prec prec, double rho, double mu, double dt,
                     const double* grav, const void* u, const void* p, void* ustar, void* ws,
                     size_t ws_bytes, void* stream);
/* Step 3, Eqs. (ns_lp1)-(ns_lp3): V = ustar / dt + G p_old / rho;         */
/* (1/rho) D G                                                              */
/* p_new = D V (Fourier modes where the symbol of D G vanishes -- the      */
/* constant and those with two or more Nyquist components -- get p_new = 0); */
/* u_new = dt (V - G p_new / rho), so D u_new = 0.  u_new may alias ustar,  */
/* p_new may alias p_old.  In FP32 the solve's own rounding would reach p  */
/* amplified by up to the condition number of D G (about n^2/pi^2), so the  */
/* residual D (V - G p1/rho) of the first solve p1 is summed in FP64 and a  */
/* second FP32 solve of it corrects p (one step of iterative refinement).   */
int ib_fluid_project(int32_t n, double h, ib_prec prec, double rho, double dt,
                     const void* ustar, const void* p_old, void* u_new, void* p_new, void* ws,
                     size_t ws_bytes, void* stream);
/* Layout moves between a global field [3][n2][n1][n0] (x fastest) and the  */
/* box layout of lv (valid cells of the covered boxes only; ghost cells of  */
/* boxed and cells of uncovered boxes in glob are left alone).              */
int ib_field_to_boxes(const ib_level* lv, ib_prec prec, const void* glob, void* boxed,
                      void* stream);
int ib_field_from_boxes(const ib_level* lv, ib_prec prec, const void* boxed, void* glob,
                        void* stream);

const char* ib_status_string(int status);
const char* ib_last_hip_error(void);
int ib_version(void);

#ifdef __cplusplus
}
#endif

#endif /* IBX_H */
