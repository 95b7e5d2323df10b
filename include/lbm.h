/*
 * lbm.h -- C ABI of the MI355X (gfx950) lattice Boltzmann library for
 * Bingham (yield-stress) fluids: fused stream-collide with the
 * Papanastasiou-regularised (PR) and implicitly-regularised (IR) operators of
 * Regulski, Leonardi & Szumbarski, "On the spatial convergence and transient
 * behaviour of lattice Boltzmann methods for modelling fluids with yield
 * stress" (arXiv:1610.01388).
 *
 * General rules
 *   - Every function is extern "C", never throws and never aborts; it
 *     returns LBM_OK (0) or a negative lbm_status.  lbm_last_error() gives a
 *     message for the last failure on the calling thread.
 *   - Device memory is allocated by the caller and bound by pointer
 *     (lbm_bind); the library never allocates or frees device memory.
 *     Sizes come from lbm_query_sizes.  Host buffers are caller-owned.
 *   - All device work is enqueued on the stream given to lbm_bind, in order.
 *     Functions that return host data synchronise that stream.
 *   - Node index n = x + nx*(y + ny*z) (x fastest).  Populations are
 *     indexed [i][n] in the library's velocity order (lbm_lattice_info).
 *   - A domain is used by one host thread at a time.
 *
 * Model (what one step computes, for every fluid node x)
 *   1. streaming (Sec. 2, Eq. 10): f_i(x) = f_i^post(x - c_i), with halfway
 *      bounce-back f_i(x) = f_opp(i)^post(x) where x - c_i is solid or lies
 *      beyond a wall face (Sec. 4.3); periodic axes wrap;
 *   2. moments rho, j, Pi (Eq. 9) of the transformed populations (Eq. 11);
 *   3. PR: strain rate from the non-equilibrium second moment with the
 *      previous step's relaxation time (Sec. 2.2 Eq. 24, Sec. 3), apparent
 *      viscosity of Eqs. 36-37 with the cut-off gamma_c, TRT collision with
 *      magic number Lambda (Sec. 2.1) and EDM body force (Sec. 2.4 Eq. 34);
 *      IR: stress solve of Sec. 3.2 (Eqs. 31, 38-40) and post-collision
 *      populations of Sec. 2.3 (Eqs. 28-29) with the force term of Eq. 35;
 *   4. store the post-collision populations (and PR's relaxation time).
 *   The reported velocity is j/rho + g/2 for both operators.
 *   Walls of non-periodic axes sit half a node outside the first and last
 *   node; solid nodes (mask byte 1) are never updated.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,    /* invalid argument or descriptor                    */
    LBM_ENOMEM = -2,    /* a bound buffer is smaller than required           */
    LBM_EHIP = -3,      /* a HIP runtime call failed                         */
    LBM_ESTATE = -4,    /* call out of order (e.g. step before bind)         */
    LBM_EUNSTABLE = -5, /* monitors found non-finite values or |u| > umax    */
    LBM_EFORMAT = -6    /* checkpoint blob malformed or for another domain   */
} lbm_status;

typedef enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1, LBM_D3Q27 = 2 } lbm_lattice;
/* LBM_PR: Papanastasiou-regularised TRT + EDM with the explicit relaxation-
 * time update (Sec. 3, 3.1: the strain rate uses the previous step's tau,
 * kept per node in the tau buffer).  LBM_IR: implicitly regularised (Sec.
 * 2.3, 3.2).  LBM_PRI: the PR model with the implicit update of Sec. 3: the
 * tau consistent with its own strain rate, found per node each step by
 * bracketed Newton iterations; nothing is kept between steps (no tau
 * buffer).  LBM_IRHB: the implicit construction of LBM_IR (Sec. 2.3, Eq.
 * 31) solved for a Herschel-Bulkley fluid, sigma = sigma_y + K g^n, as Sec.
 * 3.2 notes other laws can be: nu_p is the consistency K, hb_n the flow
 * index n (n = 1: Bingham; sigma_y = 0: power-law fluid).  With the strain
 * rate g = 3|s|/sqrt(2) the contraction of Eq. 31 gives
 * s/2 + 3 K (3/sqrt 2)^(n-1) s^n + sqrt(2) sigma_y = |dev T| for the
 * magnitude s of the collision's second moment, solved per node by
 * bracketed Newton iterations. */
typedef enum { LBM_PR = 0, LBM_IR = 1, LBM_PRI = 2, LBM_IRHB = 3 } lbm_operator;
/* Storage of the populations.  All three store deviations h_i = f_i - w_i
 * rho0.  FP64: h in double, collision in double.  FP32: h in float,
 * collision in float.  FP16: h_i * 2^k / w_i in IEEE half (k =
 * fp16_scale_log2, round to nearest even), collision in float. */
typedef enum { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16 = 2 } lbm_precision;
/* A/B: two population copies, pull streaming.  AA: one copy, streaming
 * folded into alternate steps (in place). */
typedef enum { LBM_AB = 0, LBM_AA = 1 } lbm_scheme;
/* COMPACT: population slots for fluid nodes only (numbered in node order),
 * solid mask held as one bitmap per (y, z) row; the step reads and writes
 * fluid data only.  DENSE: a slot for every node, one mask byte per node
 * staged in LDS tiles.  Both give identical results. */
typedef enum { LBM_COMPACT = 0, LBM_DENSE = 1 } lbm_layout;
/* Kernel of the compact layout's neighbour phases (the AA step that reads
 * and writes neighbours' slots, and every A/B step).  ROWS runs one
 * wavefront per 64-node row segment over the tiles of lbm_set_tile (lanes
 * of solid nodes idle; fastest when most nodes are fluid).  SLOTS runs one
 * thread per fluid slot, 64 consecutive slots per wavefront (every lane
 * busy; fastest when most nodes are solid).  AUTO (default) takes SLOTS
 * when fewer than 45% of the nodes are fluid, else ROWS.  Identical
 * results. */
typedef enum { LBM_PULL_AUTO = 0, LBM_PULL_SLOTS = 1, LBM_PULL_ROWS = 2 } lbm_pull_form;

typedef struct {
    int32_t lattice;     /* lbm_lattice                                      */
    int32_t nx, ny, nz;  /* nodes per axis; nz must be 1 for D2Q9            */
    int32_t periodic[3]; /* nonzero: periodic axis; 0: bounce-back walls     */
    int32_t precision;   /* lbm_precision                                    */
    int32_t scheme;      /* lbm_scheme                                       */
    int32_t layout;      /* lbm_layout                                       */
} lbm_desc;

typedef struct {
    int32_t op;              /* lbm_operator                                  */
    int32_t fp64_fallback;   /* FP32/FP16: redo near-yield nodes in FP64      */
    double nu_p;             /* plastic kinematic viscosity (> 0)             */
    double sigma_y;          /* yield stress per unit density (>= 0)          */
    double rho0;             /* reference density (> 0), usually 1            */
    double m;                /* PR: Papanastasiou parameter (>= 0)            */
    double gamma_c;          /* PR: strain-rate cut-off (> 0), e.g. 1e-8      */
    double lambda_trt;       /* PR: TRT magic number (> 0), e.g. 0.25         */
    double g[3];             /* body force per unit mass                      */
    double fallback_band;    /* FP64 redo (fp64_fallback) of the nodes whose
                                stress lies within this relative band around
                                the yield stress: IR |T/(sqrt2 sigma_y) - 1|
                                < band, PR and PRI |rho nu_app gamma_dot /
                                sigma_y - 1| < band (sigma_y > 0)          */
    int32_t fp16_scale_log2; /* FP16: k in h*2^k/w (0..24), e.g. 14           */
    int32_t flow_axis;       /* 0: off.  1, 2, 3: the flow is known to run along
                                x, y, z; the collision then drops that axis's
                                normal component (Sec. 4.2.2): PR leaves d_aa
                                out of the strain rate, IR sets T_aa to zero
                                before the deviator.  Other values: EINVAL. */
    double mrt_bulk;         /* PR, PRI: MRT base collision (Sec. 2.1, Eqs. 20 */
    double mrt_even;         /* and 23) instead of TRT.  Relaxation rates in
                                (0, 2) of the bulk (trace) moment and of the
                                even moments of order >= 4; 0 takes the shear
                                rate 1/tau.  Both 0: TRT.  The moment basis
                                is orthogonal under the lattice weights
                                (shear and bulk parts of the second-order
                                Hermite projection, the odd moments at the
                                magic-number rate, the rest).  IR: must be 0;
                                PRI: mrt_bulk must be 0.  Out of [0, 2):
                                EINVAL. */
    double hb_n;             /* IRHB: flow index n in [0.2, 5]; other
                                operators: ignored */
} lbm_rheology;

typedef struct {
    int64_t step;           /* time of the record (collisions done)           */
    double flux[3];         /* sum of velocity over fluid nodes / all nodes   */
    double mass;            /* sum of rho over fluid nodes                    */
    double umax;            /* max |u| over fluid nodes                       */
    int64_t fluid_nodes;
    int64_t unyielded;      /* IR: T <= sqrt2 sigma_y; PR: rho nu_app gamma_dot < sigma_y */
    int64_t fallback_nodes; /* nodes recomputed in FP64 (reduced precision)   */
    int64_t nonfinite;      /* fluid nodes with a non-finite rho or u         */
    /* Convergence towards a steady state (the velocity-change criteria of
     * Sec. 4.3 and 4.5): with u_prev each fluid node's output velocity at
     * the previous fused monitor record (zero after lbm_init_equilibrium,
     * lbm_set_mask or lbm_write_populations),
     *   residual = sum |u - u_prev|^2 / sum |u|^2   (0 when sum |u|^2 = 0),
     *   du_max   = max |u - u_prev|.
     * Fused records then store u as the next u_prev; lbm_monitors compares
     * with the last fused record's velocity and stores nothing. */
    double residual;
    double du_max;
} lbm_monitor;

typedef struct {
    size_t pdf_bytes;   /* population storage (x2 for A/B)                  */
    size_t tau_bytes;   /* PR relaxation-time field (0 for IR)             */
    size_t mask_bytes;  /* uint8 per node                                  */
    size_t work_bytes;  /* monitor partials, history ring, IO staging      */
} lbm_sizes;

typedef struct lbm_domain lbm_domain;

/* Message for the last error on this thread ("" if none). */
const char* lbm_last_error(void);

/* Library velocity order: c (3*q ints), w (q doubles), opp (q ints); any
 * pointer may be NULL.  *q receives the velocity count. */
int lbm_lattice_info(int32_t lattice, int32_t* q, int32_t* c, double* w, int32_t* opp);

/* Bytes of each device buffer the caller must bind for this descriptor. */
int lbm_query_sizes(const lbm_desc* desc, const lbm_rheology* rh, lbm_sizes* out);

/* Validate and create a domain.  Errors (LBM_EINVAL): unknown lattice,
 * precision or scheme; non-positive sizes; nz != 1 for D2Q9; nu_p <= 0;
 * sigma_y < 0; rho0 <= 0; PR with m < 0, gamma_c <= 0 or lambda_trt <= 0;
 * fp16_scale_log2 outside 0..24; fallback_band < 0; IRHB with hb_n outside
 * [0.2, 5]. */
int lbm_create(const lbm_desc* desc, const lbm_rheology* rh, lbm_domain** out);

/* Bind caller-owned device buffers (sizes from lbm_query_sizes; tau may be
 * NULL for IR) and the HIP stream (hipStream_t, NULL = default stream).
 * The mask buffer is cleared to all-fluid and the populations are set to
 * rest at rho0 (lbm_init_equilibrium(rho0, 0)). */
int lbm_bind(lbm_domain* dom, void* pdf_dev, void* tau_dev, void* mask_dev, void* work_dev,
             void* hip_stream);

/* Set the solid mask from a host array (N bytes, 1 = solid, 0 = fluid) and
 * reset the state to rest (lbm_init_equilibrium(rho0, 0)): the compact
 * layout renumbers the population slots.  Synchronises. */
int lbm_set_mask(lbm_domain* dom, const uint8_t* host_mask);

/* Post-collision state f_eq(rho0, u0) at every fluid node, time 0; PR
 * relaxation time set to the zero-strain value 1/2 + 3 (nu_p + m sigma_y/rho0)
 * (Sec. 4.4 start from rest: u0 = 0). */
int lbm_init_equilibrium(lbm_domain* dom, double rho0, const double* u0);

/* Set / get the post-collision populations of the last step (q*N doubles,
 * [i][n], library order, full f_i -- not deviations) and, for PR, the
 * relaxation-time field (N doubles; may be NULL).  Writing converts to the
 * storage precision.  Both synchronise. */
int lbm_write_populations(lbm_domain* dom, const double* host_P, const double* host_tau);
int lbm_read_populations(lbm_domain* dom, double* host_P, double* host_tau);

/* Enqueue nsteps time steps (asynchronous).  With graph steps G > 0 (see
 * lbm_set_graph_steps), runs of G steps that start at a time that is a
 * multiple of G, from the post-collision state in the first copy (A/B) or the
 * even AA phase, replay one captured hipGraph of G launches; the other steps
 * launch eagerly.  Results are identical either way. */
int lbm_step(lbm_domain* dom, int64_t nsteps);
/* Steps per captured graph (even, >= 0; 0, the default, launches every step
 * eagerly).  The graph is captured on first use on a private stream of the
 * default priority and captured again after any change to what the launches
 * carry (tile, tile order, neighbour-phase kernel, mask, monitor interval,
 * checkpoint load).  It pays for small domains, whose steps are short enough
 * for the launch overhead to matter.  With monitors, G must be a multiple of
 * the monitor interval for replays to be used.  LBM_EINVAL for an odd or
 * negative count. */
int lbm_set_graph_steps(lbm_domain* dom, int32_t steps);

/* Current time (number of collisions done). */
int lbm_time(lbm_domain* dom, int64_t* t);

/* Fuse monitors into every k-th step (0 = off).  Each record (lbm_monitor of
 * the state the step starts from) goes to a device ring of 4096 records;
 * lbm_read_history copies out the records produced since the last call
 * (oldest first, at most max) and synchronises. */
int lbm_set_monitor_interval(lbm_domain* dom, int32_t k);
int lbm_read_history(lbm_domain* dom, lbm_monitor* out, int32_t max, int32_t* count);

/* Monitors of the current state; synchronises.  Returns LBM_EUNSTABLE (with
 * *out filled) when a fluid node is non-finite or umax exceeds the limit set
 * by lbm_set_umax_limit (default 0.1, the Mach validity bound of Sec. 4.5.3). */
int lbm_monitors(lbm_domain* dom, lbm_monitor* out);
int lbm_set_umax_limit(lbm_domain* dom, double umax);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * monitors of the current state, as lbm_monitors computes them (residual
 * against the last fused record, nothing stored), written as one lbm_monitor
 * into caller-owned device memory record_dev (8-byte aligned), enqueued on
 * the bound stream without synchronising.  Its kernels keep their per-block
 * partial sums in a per-GPU file-scope device array of 2048 x 12 doubles
 * (192 KiB, held by each GPU the library runs on until the process ends), not
 * in the bound work buffer; the reduction runs at most 2048 blocks (a grid
 * stride over the nodes), so every domain size fits.  lbm_bind resolves the
 * array's address on the bound stream's GPU, so this call does no symbol
 * lookup: it enqueues two kernels.  Nothing is allocated,
 * freed or cleared: every block overwrites its own partials.  Calls that
 * overlap on one GPU (other streams or threads) race on that array and must
 * be serialised by the caller.  No LBM_EUNSTABLE check: the record carries
 * nonfinite and umax.  LBM_EINVAL for a NULL or misaligned record_dev. */
int lbm_monitors_async(lbm_domain* dom, void* record_dev);

/* Moments of the current state into host buffers (N doubles rho, 3*N
 * doubles u component-major u[a*N+n], N doubles nu_app (PR; IR reports
 * nu_p), N bytes unyielded flag).  Any pointer may be NULL.  Solid nodes
 * report zeros.  Synchronises. */
int lbm_read_moments(lbm_domain* dom, double* rho, double* u, double* nu_app,
                     uint8_t* unyielded);

/* Checkpoint.  The blob is a header followed by the payload:
 *   header: magic "LBMCKPT1", format version 3, header size, the domain's
 *     lbm_desc and lbm_rheology, the time (collisions done), the population
 *     stride, the fluid count, the AA phase (0: post-collision state, 1:
 *     streamed state; always 0 for A/B), q, the four payload part sizes and a
 *     checksum of the payload (FNV-1a over 64-bit words in four interleaved
 *     lanes);
 *   payload: the raw population storage (q x stride elements of the storage
 *     precision), the PR relaxation-time field (stride elements; absent for
 *     the other operators), the mask (dense layout: N bytes, 1 = solid;
 *     compact layout: the fluid bitmap, ny nz rows of ceil(nx / 64) 64-bit
 *     words, bit b of word w set when node x = 64 w + b is fluid) and the
 *     residual monitor's reference velocity (3 x stride doubles).
 * With blob == NULL, lbm_save only reports the size in *bytes.  lbm_load
 * validates the whole blob on the host before any device work and rejects
 * it (LBM_EFORMAT) when it is truncated, saved from another descriptor, fails
 * its checksum, or is inconsistent: a negative time, an AA phase outside
 * {0, 1}, a mask byte other than 0 / 1, a fluid bit past a row's end, a fluid
 * count or stride that the mask does not give.  The slot tables of the
 * compact layout are rebuilt from the mask, never read from the blob.  The
 * rheology in the blob is informational: the domain keeps its own (a state
 * may be continued under other rheological parameters).  Both synchronise. */
int lbm_save(lbm_domain* dom, void* blob, size_t* bytes);
int lbm_load(lbm_domain* dom, const void* blob, size_t bytes);
/* The validation lbm_load performs, for a domain of this descriptor and
 * rheology, on the host alone (no device, no domain needed): LBM_OK or
 * LBM_EFORMAT (LBM_EINVAL for an invalid descriptor or rheology). */
int lbm_check_checkpoint(const lbm_desc* desc, const lbm_rheology* rh, const void* blob, size_t bytes);

/* Tile shape of the step kernel: one node per thread, tx*ty*tz threads per
 * block, which must be 64, 128, 192 or 256; tz must be 1 for D2Q9; the
 * compact layout needs tx = 64, 128 or 256 (one wavefront per 64-node row
 * segment; wider tiles hold adjacent segments of a row in one block). */
int lbm_set_tile(lbm_domain* dom, int32_t tx, int32_t ty, int32_t tz);
int lbm_get_tile(lbm_domain* dom, int32_t* tx, int32_t* ty, int32_t* tz);
/* Order in which the step walks its tiles: bricks of whole rows x
 * brick_rows tile rows x brick_planes tile planes (x fastest, then y, then
 * z inside a brick), so that tiles that touch the same cache lines across
 * z run close together and on one XCD.  0 selects the default (compact
 * layout: about 16 tiles per brick plane and one slab of planes per XCD;
 * dense layout: one brick, i.e. plain x, y, z order); values are clamped to
 * the tile grid.  The order changes timing only, never results.  The getter
 * reports the values in effect. */
int lbm_set_tile_order(lbm_domain* dom, int32_t brick_rows, int32_t brick_planes);
int lbm_get_tile_order(lbm_domain* dom, int32_t* brick_rows, int32_t* brick_planes);
/* Select the compact layout's neighbour-phase kernel (lbm_pull_form); tiles
 * and tile order apply to ROWS only.  LBM_EINVAL for another value.  The
 * dense layout ignores the setting.  Timing only, never results.  The
 * getter reports the kernel in effect (SLOTS or ROWS; AUTO resolved with
 * the current mask). */
int lbm_set_pull_form(lbm_domain* dom, int32_t form);
int lbm_get_pull_form(lbm_domain* dom, int32_t* form);
/* Time candidate tile shapes (compact layout: and both neighbour-phase
 * kernels) on the bound buffers (the state is saved and restored around the
 * trial steps) and keep the fastest; synchronises. */
int lbm_autotune(lbm_domain* dom, int32_t trial_steps);

int lbm_destroy(lbm_domain* dom);

/* ---------------------------------------------------------------------------
 * Batched sweep: count independent simulations of uneven size (for example
 * the square ducts of a Bingham-number sweep, Sec. 4.3) advanced together.
 * Every simulation is all-fluid inside its box (walls only through
 * non-periodic axes) and has its own sizes, operator and rheology; all
 * share one lattice, one precision, the AA scheme, the FP64-fallback flag
 * and the FP16 scale; each holds fewer than 2^31 / Q nodes and uses LBM_PR
 * or LBM_IR.  One step is one persistent kernel launch over a work
 * list of 256-node items of all simulations (runs of consecutive nodes,
 * or 3-D tiles, per lbm_batch_set_schedule); lbm_batch_step replays a
 * captured hipGraph of graph_steps such launches when it can.  The update
 * of each node is the same as lbm_step's (a simulation gives bitwise the
 * same state batched or alone).
 * ------------------------------------------------------------------------- */
typedef struct lbm_batch lbm_batch;

/* Device bytes for the arena (pdf), relaxation times (tau, 0 without PR)
 * and the work buffer (parameter table, work list, monitors, staging);
 * mask_bytes is 0. */
int lbm_batch_query_sizes(const lbm_desc* descs, const lbm_rheology* rh, int32_t count, lbm_sizes* out);
/* Validate (as lbm_create for each, plus the shared-field rules above) and
 * plan the work list. */
int lbm_batch_create(const lbm_desc* descs, const lbm_rheology* rh, int32_t count, lbm_batch** out);
/* Bind caller-owned device buffers and the stream; uploads the parameter
 * table and work list and sets every simulation to rest. */
int lbm_batch_bind(lbm_batch* b, void* pdf_dev, void* tau_dev, void* work_dev, void* hip_stream);
int lbm_batch_init_equilibrium(lbm_batch* b);
/* Per-simulation population I/O and readout, as the single-domain calls
 * (writes are allowed at even times only); synchronise. */
int lbm_batch_write_populations(lbm_batch* b, int32_t sim, const double* host_P, const double* host_tau);
int lbm_batch_read_populations(lbm_batch* b, int32_t sim, double* host_P, double* host_tau);
int lbm_batch_read_moments(lbm_batch* b, int32_t sim, double* rho, double* u, double* nu_app, uint8_t* unyielded);
/* Fused per-simulation monitors every k steps into a device ring of 256
 * records per simulation; lbm_batch_read_history copies records (each
 * record = count lbm_monitor, one per simulation) produced since the last
 * call, at most max_records of them, and synchronises. */
int lbm_batch_set_monitor_interval(lbm_batch* b, int32_t k);
int lbm_batch_read_history(lbm_batch* b, lbm_monitor* out, int32_t max_records, int32_t* nrecords);
/* Monitors of every simulation's current state (count records). */
int lbm_batch_monitors(lbm_batch* b, lbm_monitor* out);
/* Steps per captured graph (even; 0 = always launch eagerly; default 100).
 * A replay starts at times that are multiples of it; other steps are
 * launched eagerly. */
int lbm_batch_set_graph_steps(lbm_batch* b, int32_t steps);
int lbm_batch_step(lbm_batch* b, int64_t nsteps);
int lbm_batch_time(lbm_batch* b, int64_t* t);
/* Tile shape chosen for each simulation (3*count ints). */
int lbm_batch_get_tiles(lbm_batch* b, int32_t* tiles);
/* Scheduling in use: tile policy (0 fewest padded nodes, 1 rows at least
 * 64 wide, 2 fixed 64x4x1, 3, the default, runs of 256 consecutive nodes in
 * node order, rows wrapping, reported by lbm_batch_get_tiles as 256x1x1) and
 * work-item order (0, the default, plain grid stride over the list; 1 one
 * contiguous chunk of the list per XCD so that neighbouring tiles share an
 * L2). */
int lbm_batch_get_schedule(lbm_batch* b, int32_t* tile_policy, int32_t* xcd_order);
/* Choose the scheduling by hand (the state is kept; results do not depend on
 * it).  LBM_EINVAL outside the ranges above.  Synchronises. */
int lbm_batch_set_schedule(lbm_batch* b, int32_t tile_policy, int32_t xcd_order);
/* Time every tile policy with both work-item orders on trial_steps steps of
 * the bound batch and keep the fastest; the state is restored.  The device
 * layout does not depend on the choice.  Synchronises. */
int lbm_batch_autotune(lbm_batch* b, int32_t trial_steps);
int lbm_batch_destroy(lbm_batch* b);

#ifdef __cplusplus
}
#endif
#endif
