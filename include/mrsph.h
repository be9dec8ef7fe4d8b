/*
 * mrsph: multi-resolution SPH for fluid-structure interaction on AMD Instinct
 * MI355X (gfx950).  The method is that of Zhang, Rezavand & Hu,
 * "A multi-resolution SPH method for fluid-structure interactions"
 * (arXiv:1911.13255): a weakly-compressible fluid at smoothing length h_F,
 * a total-Lagrangian elastic solid at h_S <= h_F integrated kappa times per
 * fluid acoustic step, and a coupling force built from the solid's
 * time-averaged velocity and acceleration inside a position-based Verlet
 * scheme (Algorithm 1).
 *
 * Conventions for every entry point below:
 *  - Return value: SPH_OK (0), a negative SPH_E_* error, or a positive info
 *    code.  No C++ exception crosses this interface.
 *  - Asynchrony: calls that advance the simulation only enqueue kernels on the
 *    context's stream.  Errors raised inside kernels (NaN, inverted solid
 *    element, neighbour-capacity overflow) are latched in device memory and
 *    reported by sph_sync and by sph_read/sph_scalars, which synchronise.
 *  - Memory: all device memory is one caller-owned arena of sph_arena_bytes()
 *    bytes (e.g. a uint8 tensor).  The library never allocates or frees device
 *    memory; sph_init allocates the host context and a small pinned host
 *    buffer (the scene states, read back asynchronously by the streamed
 *    solid passes), and sph_destroy frees both.
 *  - Host arrays passed in are read during the call only.
 *  - Threading: one context per stream; calls on one context are not
 *    thread-safe.  Contexts are independent.
 *  - Order (Algorithm 1): one acoustic step is neighbor_build, fluid_step,
 *    couple, solid_substeps, in this order (neighbor_build rebuilds only the
 *    scenes whose advection step is due, and may be repeated).  A context
 *    starts at a step boundary; sph_advance, sph_write, sph_set_scalars,
 *    sph_set_surrogate, sph_solid_targets and sph_time_kernel run only
 *    there; sph_solid_features only between couple and solid_substeps.  A
 *    call out of this sequence returns SPH_E_ORDER, enqueues nothing and
 *    leaves the state and the sequence as they were.  Read-only calls
 *    (sph_read, sph_reduce, sph_pairs, counters, scalars) run anywhere in it.
 *  - Units are SI; positions are row-major (n, dim) float64.
 */
#ifndef MRSPH_H
#define MRSPH_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPH_OK 0
#define SPH_E_ARG (-1)      /* invalid argument or scene description */
#define SPH_E_HIP (-2)      /* a HIP runtime call failed */
#define SPH_E_ORDER (-3)    /* call out of sequence (e.g. before sph_init) */
#define SPH_E_CAPACITY (-4) /* a fixed-capacity neighbour table or pair list overflowed */
#define SPH_E_UNSTABLE (-5) /* NaN/Inf in the state or det F <= 0 (reported first when both hold) */
#define SPH_FALLBACK 1      /* info (sph_sync): a learned sub-step fell back to the plain sub-steps
                               since the previous sph_sync */

typedef struct sph_ctx sph_ctx;

/* One scene.  Fluid, wall and solid particle sets with their materials.
 * Solid particles are free ones first; the last n_clamp form the rigid base
 * block that holds the structure (u = 0, v = 0, F = I at all times). */
typedef struct {
  int dim;                               /* 2 or 3; all scenes of a context share it */
  int n_fluid, n_wall, n_solid, n_clamp; /* particle counts */
  double dp_f, dp_s, h_ratio;            /* spacings; h = h_ratio * dp (1.3 in the paper) */
  double rho0_f, c_f, eta, gamma;        /* fluid reference density, sound speed, dynamic viscosity, Tait exponent */
  double g[3];                           /* body acceleration */
  double rho0_s, E, nu;                  /* solid density, Young's modulus, Poisson ratio */
  double cfl_ac, cfl_ad, cfl_s, u_ref;   /* acoustic, advection and solid CFL numbers; velocity floor of dt_ad */
  double lo[3], hi[3];                   /* cell-grid box; particles outside it stay valid */
  int periodic[3];                       /* periodic axes (box length = hi - lo; >= 3 cells of 2 h_F) */
  double hydro_H;                        /* initial hydrostatic surface height along the last axis */
  double inflow_U0, inflow_ts, inflow_H, inflow_len; /* inflow buffer (inflow_len = 0: none) */
  const double *x_fluid, *v_fluid;       /* (n_fluid, dim); v_fluid may be NULL */
  const double *x_wall, *nrm_wall;       /* (n_wall, dim): wall positions and unit normals into the fluid */
  const double *x_solid, *v_solid;       /* (n_solid, dim); v_solid may be NULL */
  int material;    /* solid law (Section 2.1): 0 Neo-Hookean, 1 linear elastic in the
                      Green-Lagrange strain, S = lambda tr(E) I + 2 mu E (Kirchhoff) */
  int single_step; /* 0: multiple time steps, kappa = floor(dt_ac / dt_S) + 1 solid
                      sub-steps per acoustic step (Section 3.2); 1: the contrast the
                      same section names, dt_S (when smaller) as the one step of fluid
                      and structure, kappa = 1 */
} sph_scene;

typedef struct {
  int riemann;        /* 1: low-dissipation Riemann solver (Section 2.2); 0: simple averages */
  int density_reinit; /* 0 off; 1 rho = rho0 max(1, psi/psi0); 2 rho = max(rho, rho0 psi/psi0) */
  int max_solid_nbr;  /* capacity of the solid reference neighbour table; 0 = default (40 in 2D, 128 in 3D) */
  int solid_block;    /* threads per scene of the register-resident solid kernel (power of two, 64..1024); 0 = default */
  int lanes_per_particle; /* lanes sharing one particle in the fluid pair loops (1, 2, 4, 8, 16); 0 = chosen from the particle count */
  int block_pair;     /* threads per block of the fluid pair loops (64, 128, 256); 0 = default */
  int solid_lds;      /* 0: 2D scenes whose free solid fits 2048 particles run one register-resident
                         kernel per step (v and P B in LDS), other solids streamed passes;
                         1: always the streamed passes */
  int max_fluid_nbr;    /* capacity of each fluid particle's fluid pair list; 0 = default (twice the
                           lattice count inside 2 h_F) */
  int max_boundary_nbr; /* capacity of each fluid particle's wall and solid pair list; 0 = default
                           (lattice count inside 2 h_F times 1 + (dp_F/dp_S)^d) */
  int serial_passes;    /* 0: in sph_advance the continuity pass runs on a second stream,
                           concurrently with the coupling and solid passes; 1: one stream */
  int solid_parts;      /* 0: the register-resident solid kernel runs one workgroup per scene;
                           > 0: on serial steps without a surrogate, a scene with more free solid
                           particles than this runs on ceil(n / solid_parts) workgroups (at most
                           256 in all; scenes with one shared step keep one), which exchange
                           P B and v through global memory between the half sub-steps.  Results
                           equal the one-workgroup form bit for bit; it measured slower on the
                           channel and the batch, so 0 is the default and the autotuner keeps
                           the caller's value */
  int fluid_tiles;      /* 0: in 3D, each block of the fluid force and continuity passes stages the
                           records of its particles' distinct fluid neighbours (at most 768) in LDS
                           and reads them there; the rebuild writes a second, 16-bit copy of those
                           particles' fluid rows that indexes that set (2 bytes per pair-list slot
                           more device memory).  Results equal the per-pair gathers bit for bit.
                           -1: per-pair gathers.  2D always uses per-pair gathers. */
  int solid_blocks;     /* 0: in 3D, where every scene's solid sits near one lattice (each particle
                           within a quarter spacing of its own lattice point, a bounding box of at
                           most 4 cells per particle) and its reference neighbours are exactly the
                           lattice points at offsets that reach within 2 h_S, the streamed sub-step
                           passes run one workgroup per block of 4 x 4 x 16 lattice cells: it stages
                           the P B or v of the cells within two spacings in LDS and sums over the
                           offset classes in place of the pair table.  On an exact lattice (the
                           compact table) a class carries its gradient; otherwise each pair's
                           gradient is formed in FP32 from the class's lattice vector and the two
                           particles' offsets (all scenes with solid then of one spacing,
                           smoothing length and volume).  16 bytes per cell of the bounding boxes
                           more device memory.  Sums run in class order, not table order, so
                           results differ from the table walk by FP32 rounding.  -1: the pair
                           table. */
} sph_options;

/* Field ids for sph_read / sph_write (FP64, original particle order).
 * Vectors are (n, dim), tensors (n, dim, dim) row-major. */
enum {
  SPH_F_X = 0,    /* fluid position */
  SPH_F_V = 1,    /* fluid velocity */
  SPH_F_RHO = 2,  /* fluid density */
  SPH_F_DRHO = 3, /* fluid density rate kept for the next half step */
  SPH_F_A = 4,    /* fluid acceleration of the last step (read only) */
  SPH_F_P = 5,    /* fluid mid-step pressure of the last step (read only) */
  SPH_F_NNB = 6,  /* (fluid, wall + solid) neighbours within 2 h_F at the last rebuild (read only) */
  SPH_S_U = 10,   /* solid displacement */
  SPH_S_V = 11,   /* solid velocity */
  SPH_S_A = 12,   /* solid acceleration of the last sub-step */
  SPH_S_F = 13,   /* deformation gradient */
  SPH_S_DF = 14,  /* rate of the deformation gradient */
  SPH_S_FF = 15,  /* force from the fluid (read only) */
  SPH_S_VBAR = 16,/* time-averaged velocity over the last acoustic step */
  SPH_S_ABAR = 17,/* time-averaged acceleration over the last acoustic step */
  SPH_S_N = 18,   /* current surface normal (read only) */
  SPH_S_B = 19,   /* correction matrix (read only) */
  SPH_S_N0 = 20,  /* reference surface normal (read only) */
  SPH_S_X0 = 21   /* reference position (read only) */
};

/* Bytes of device memory needed by sph_init for these scenes and options;
 * 0 on invalid input. */
size_t sph_arena_bytes(const sph_scene *scenes, int n_scenes, const sph_options *opt);

/* Set up the scenes (Algorithm 1, before the time loop): fluid state with a
 * hydrostatic initial density, reference configuration of the solid with its
 * neighbour table, FP64 correction matrices B and reference normals.
 * dev_arena: device pointer to arena_bytes >= sph_arena_bytes() bytes, owned
 * by the caller and kept alive until sph_destroy.  stream: a hipStream_t
 * (NULL selects the null stream, which sph_advance cannot graph-capture).
 * On success *out holds the new context.  Synchronises before returning. */
int sph_init(const sph_scene *scenes, int n_scenes, const sph_options *opt, void *dev_arena,
             size_t arena_bytes, void *stream, sph_ctx **out);

/* Start of an advection step where one is due, per scene (Algorithm 1, outer
 * loop; Section 3.2, advection criterion): advection time step, cell-linked
 * lists (Morton-ordered counting sort of the fluid and of walls + solid into
 * cells of 2 h_F), frozen pair geometry, density reinitialisation, update of
 * the solid surface normals.  Scenes with no advection step due are left as
 * they are.  Enqueue only. */
int neighbor_build(sph_ctx *ctx);

/* One fluid acoustic step of the position-based Verlet scheme (Section 3.3):
 * half step in density and position, momentum with the Riemann pressure,
 * viscous and coupling forces at h_F (Section 3.1), full step in velocity,
 * continuity with the new velocity, second half step.  Must follow
 * neighbor_build (else SPH_E_ORDER).  Enqueue only. */
int fluid_step(sph_ctx *ctx);

/* Pressure and viscous forces of the fluid on the solid (Section 2.2,
 * Eqs. F:p and F:v at h_F), as exact negatives of the fluid-side pair terms
 * of the same step.  Must follow fluid_step (else SPH_E_ORDER).  Enqueue
 * only. */
int couple(sph_ctx *ctx);

/* kappa solid sub-steps of the position-based Verlet scheme with the fluid
 * force held constant (Section 3.3), Neo-Hookean stress (Section 2.1) and
 * the corrected total-Lagrangian momentum equation at h_S (Section 3.1);
 * then the time-averaged velocity and acceleration (Section 3.2) and the
 * end-of-step time bookkeeping.  Must follow couple (else SPH_E_ORDER).
 * Enqueue only, except
 * for solids run as streamed passes (3D, large or solid_lds = 1): there
 * kappa is read back to the host, which waits for the stream. */
int solid_substeps(sph_ctx *ctx);

/* n acoustic steps of Algorithm 1 (neighbor_build, fluid_step, couple,
 * solid_substeps); the first call captures one step into a HIP graph that
 * later calls replay.  Enqueue only.  With streamed solid passes the steps
 * are launched one by one without a graph and each waits for kappa. */
int sph_advance(sph_ctx *ctx, int n_steps);

/* Copy a field of one scene to host memory in original particle order
 * (FP64).  host must hold n * (1 | dim | dim*dim) doubles.  Synchronises. */
int sph_read(sph_ctx *ctx, int field, int scene, double *host);

/* Overwrite a state field of one scene from host memory (FP64, original
 * order).  Writing positions or velocities marks the scene for a rebuild at
 * the next neighbor_build.  Synchronises. */
int sph_write(sph_ctx *ctx, int field, int scene, const double *host);

/* Scene time state: out[0..7] = t, dt_ac, dt_ad, dt_s, adv_accum, kappa,
 * need_rebuild, max fluid speed.  Synchronises. */
int sph_scalars(sph_ctx *ctx, int scene, double *out);

/* Overwrite t, dt_ad, adv_accum and need_rebuild of one scene from
 * in[0], in[2], in[4], in[6] (the other entries are ignored).  Synchronises. */
int sph_set_scalars(sph_ctx *ctx, int scene, const double *in);

/* Counters of one scene (scene = -1: sum over scenes): out[0..7] =
 * fluid-fluid pairs, fluid-wall pairs, fluid-solid pairs (of the last
 * rebuild, totalled when the acoustic step that began with it ends), solid
 * reference pairs, acoustic steps, rebuilds, solid sub-steps, particle
 * interactions evaluated.  Synchronises. */
int sph_counters(sph_ctx *ctx, int scene, unsigned long long *out);

/* Autotuner of the launch shapes (batched scenes, hipGraph replay): for
 * every candidate, lanes per fluid particle in {1, 2, 4, 8, 16} x threads
 * per block of the pair passes in {64, 128, 256} x serial_passes in {0, 1},
 * twice: initialises the scenes in the caller's arena on the caller's
 * stream, advances `warmup` acoustic steps and times `steps` more with HIP
 * events; the faster repetition counts (a trial never runs the scenes past
 * warmup + steps steps).
 * *best receives *opt with the fastest candidate's three fields; ms_per_step
 * (may be NULL) its time per step.  The arena must hold sph_arena_bytes for
 * *opt (the candidates do not change the size).  Synchronises; no context is
 * left behind.  Returns SPH_E_ARG for bad arguments, else the first error of
 * a candidate run. */
int sph_autotune(const sph_scene *scenes, int n_scenes, const sph_options *opt, void *dev_arena,
                 size_t arena_bytes, void *stream, int warmup, int steps, sph_options *best,
                 double *ms_per_step);

/* ---- learned sub-step surrogate (2D, register-resident solid kernel) ----
 * A network of include/mrsph_mlp.h with 24 inputs and 4 outputs replaces
 * the kappa solid sub-steps of acoustic steps, scene by scene, while the
 * plain sub-steps judge it.  For a free solid particle with own values
 * F - I (4, row-major), v (2), a (2) and the pressure and viscous parts
 * fp, fv (2 + 2) of the coupling force, their means over its reference
 * neighbours (the own values where it has none), the acceleration scale
 * s = |a| + |mean a| + |g| + |fp + fv| / m + 1e-3 m/s^2 (m = rho0_S V_S) and
 * the acoustic step dt, the features are, in order: F - I, v, a / s,
 * fp / (m s), fv / (m s), then the neighbour mean minus the own value of
 * each of the 12 (F's as is, v's divided by s dt, a's by s, the forces' by
 * m s).  The outputs are (vbar - v) / (s dt) (2) and (abar - a) / s (2): the
 * scaled changes of the time-averaged velocity and acceleration of Section
 * 3.2.  Per scene, each acoustic step is one of:
 *   judge step: the plain sub-steps run and stand; the network's averages
 *     are compared with theirs over the N free particles,
 *       R = max(|vbar_net - vbar|_2 / (|vbar|_2 + |g| dt sqrt(N)),
 *               |abar_net - abar|_2 / (|abar|_2 + |g| sqrt(N))),
 *     and R <= threshold opens a window of every - 1 learned steps, while
 *     R > threshold is followed by every - 1 plain steps;
 *   learned step: the sub-steps are skipped and the predicted averages
 *     advance the solid (u += dt vbar, v += dt abar, F from the corrected
 *     gradient of vbar, the stored acceleration := abar);
 *   plain step: the plain sub-steps, no network.
 * The first step after sph_set_surrogate is a judge step.  Exact averages
 * give R = 0, so they pass any threshold; a non-finite R fails every one,
 * and threshold = +infinity passes every judge whose R is finite. */
struct mlp_ctx;

/* Use `net` (kept by the caller, max_rows >= all solid particles) with the
 * standardisation stats (host, 56 floats: feature mean[24], feature 1/std[24],
 * output mean[4], output std[4]), the judge threshold and the judge interval
 * `every` (>= 1; 1 judges every step, so no step is learned); net = NULL or
 * threshold <= 0 turns the surrogate off.  The next sph_advance captures a
 * new graph.  SPH_E_ARG for 3D, streamed solids, mismatched sizes or every
 * outside [1, 2^20].  Synchronises. */
int sph_set_surrogate(sph_ctx *ctx, struct mlp_ctx *net, const float *stats, float threshold, int every);

/* Training data: features of every solid particle at the current state
 * (rows in solid order, scene after scene, 24 floats each, clamp rows zero),
 * standardised with stats_dev (device, 48 floats: mean, 1/std) or raw when it
 * is NULL; call between couple and solid_substeps.  Enqueue only. */
int sph_solid_features(sph_ctx *ctx, const float *stats_dev, float *x_dev);

/* Targets after solid_substeps of the step whose features sph_solid_features
 * took (it keeps each row's s, dt, v and a): rows of ((vbar - v) / (s dt),
 * (abar - a) / s), 4 floats each, clamp rows zero.  SPH_E_ORDER when no
 * sph_solid_features ran in this step.  Enqueue only. */
int sph_solid_targets(sph_ctx *ctx, float *t_dev);

/* Surrogate steps of one scene (scene = -1: all) since sph_init: out[0]
 * acoustic steps the network took (learned steps), out[1] steps the plain
 * sub-steps took while a network was set (judge and plain steps), out[2]
 * judge steps passed, out[3] judge steps failed.  Synchronises. */
int sph_surrogate_counters(sph_ctx *ctx, int scene, unsigned long long *out);

/* The residual R of the scene's last judge step (NaN before the first one
 * since sph_set_surrogate, and for a non-finite residual).  SPH_E_ARG for a
 * scene out of range.  Synchronises. */
int sph_surrogate_residual(sph_ctx *ctx, int scene, double *out);

/* Launch configuration chosen at sph_init (no GPU work): out[0..9] = lanes
 * per fluid particle in the pair passes, lanes per solid particle in the
 * coupling pass, threads per block of the pair passes, solid particles per
 * thread of the register-resident solid kernel (0: streamed passes),
 * threads per workgroup of that kernel, fluid and boundary pair-list
 * capacity per particle, 1 when sph_advance replays a captured HIP graph (0
 * before the first sph_advance or without a graph), the split form's target
 * of free solid particles per workgroup (0: one workgroup per scene) and its
 * workgroups. */
int sph_launch_config(sph_ctx *ctx, int *out);

/* Reference neighbour table of the solid (Section 2.2: the gradients
 * V_b grad_a W(X_a - X_b) are fixed in the reference configuration), as set
 * up by sph_init (no GPU work): out[0] = 1 when the 3D streamed sub-step
 * passes walk the compact table (every scene's solid is a lattice of one
 * spacing, smoothing length and volume, so a pair's gradient depends only on
 * its lattice offset: 4 bytes per pair, the neighbour's index and the
 * offset's class), 0 for the full table (16 bytes per pair: the FP32
 * gradient and the index); out[1] = pair capacity per solid particle;
 * out[2] = bytes per pair that the table walk reads; out[3] = lattice
 * blocks of the 3D streamed passes (sph_options.solid_blocks; 0 when they
 * walk the table; with out[0] = 0 they form each pair's gradient from its
 * lattice vector and offsets), out[4] = offset classes those blocks sum over.
 * SPH_E_ORDER without a context, SPH_E_ARG for a null out. */
int sph_solid_table(sph_ctx *ctx, int *out);

/* Neighbour tiles of the fluid force and continuity passes (Section 3.1 pair
 * sums; sph_options.fluid_tiles) as the last rebuild left them, five values:
 * out[0] particles per group, one block of the pair launches (0: no tiles),
 * out[1] groups, out[2] groups whose fluid rows index their tile (the others
 * straddle scenes or have more than 768 distinct fluid neighbours and gather
 * per pair), out[3] distinct fluid neighbours summed over those groups,
 * out[4] the largest such tile.  Waits for the context's stream (a device to
 * host copy).  SPH_E_ORDER without a context, SPH_E_ARG for a null out,
 * SPH_E_HIP on a failed copy. */
int sph_fluid_tiles(sph_ctx *ctx, long long *out);

/* FP64 reductions of one scene: out[0..2] fluid momentum, out[3..5] solid
 * momentum, out[6] fluid kinetic energy, out[7] solid kinetic energy,
 * out[8] solid strain energy, out[9..11] sum of the fluid force on the solid,
 * out[12..14] sum of the solid force on the fluid re-evaluated from the last
 * fluid step's mid-point state (valid between couple and solid_substeps).
 * Synchronises. */
int sph_reduce(sph_ctx *ctx, int scene, double *out);

/* The reductions of sph_reduce for callers that cannot allocate or
 * synchronise (code under HIP graph capture, tight serving loops): enqueue
 * only, no allocation and no host transfer.  The 16 FP64 totals (out[0..14]
 * as sph_reduce's, out[15] unused) go to out_dev, caller-owned device memory
 * of 16 doubles.  The block partials live in a static device array of the
 * library (one per GPU, kept until the process ends) instead of the arena;
 * every block writes its own partials, so nothing needs clearing between
 * calls.  blocks: 0 = one per 256 particles of the scene, at most 1024; a
 * larger count returns SPH_E_ARG (the scratch holds 1024 blocks' partials).
 * Calls that overlap on one GPU (several streams or contexts at once) race
 * on that array; calls ordered on one stream do not. */
int sph_reduce_noalloc(sph_ctx *ctx, int scene, int blocks, double *out_dev);

/* Kernel ids for sph_time_kernel. */
enum {
  SPH_K_FLUID_FORCE = 0, /* momentum pass of fluid_step */
  SPH_K_CONTINUITY = 1,  /* continuity pass of fluid_step */
  SPH_K_COUPLE = 2,      /* couple */
  SPH_K_SOLID = 3,       /* solid_substeps */
  SPH_K_REBUILD = 4      /* neighbor_build with a rebuild forced in every scene */
};

/* Average duration in milliseconds of `reps` back-to-back launches of one
 * kernel (or, for SPH_K_REBUILD, of the whole rebuild sequence) on the
 * context's stream, from two HIP events around them.  The launches are
 * captured into a HIP graph that is replayed twice, the first time untimed
 * (on the null stream, and for the streamed solid form, which reads kappa
 * back, they are launched directly).  For profiling: every launch advances
 * the state like the entry point that owns the kernel.  Synchronises. */
int sph_time_kernel(sph_ctx *ctx, int kernel, int reps, double *avg_ms);

/* Neighbour lists of one scene at the last rebuild, for checking the cell
 * search against a brute-force search (Algorithm 1, rebuild at the start of
 * each advection step; the solid's reference lists of Section 2.2).  Rows are
 * in original particle order and each row is sorted ascending (a list is a
 * set: the kernels' own order is the cell walk's).
 *   which 0: fluid -> fluid neighbours within 2 h_F (original fluid index);
 *   which 1: fluid -> boundary neighbours within 2 h_F, boundary index =
 *            wall index for walls, n_wall + free solid index for the solid;
 *   which 2: free solid -> fluid neighbours within 2 h_F (the coupling list);
 *   which 3: solid -> solid reference neighbours within 2 h_S (solid index).
 * start (host, rows + 1 ints; rows = n_fluid, n_fluid, free solid, solid) is
 * always filled; idx (host, as many ints as the return value) is filled when
 * not NULL, so a first call with idx = NULL sizes the second.  Returns the
 * number of entries (>= 0) or an error.  Synchronises; for tests and
 * diagnostics (it copies the scene's lists to the host). */
int sph_pairs(sph_ctx *ctx, int which, int scene, int *start, int *idx);

/* Wait for the stream; return the first latched device error, if any, else
 * SPH_FALLBACK when a learned step fell back since the last call, else
 * SPH_OK.  The errors: SPH_E_UNSTABLE (non-finite state, det F <= 0),
 * SPH_E_CAPACITY (a table or list overflowed), SPH_E_HIP (the workgroups of
 * a scene split over several were not resident together, so their exchange
 * gave up waiting), SPH_E_ORDER (fewer streamed sub-step passes than kappa). */
int sph_sync(sph_ctx *ctx);

/* Text of the last error of this context (static storage of the context). */
const char *sph_last_error(const sph_ctx *ctx);

/* Release the host context.  The arena stays the caller's. */
void sph_destroy(sph_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* MRSPH_H */
