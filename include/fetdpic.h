/*
 * fetdpic.h — C-ABI of the MI355X charge-conserving relativistic FETD-PIC
 * particle step (2-D, unstructured triangles, Whitney forms).
 *
 * Method: Na, Moon, Omelchenko, Teixeira, "Relativistic extension of a
 * charge-conservative finite element solver for time-dependent
 * Maxwell-Vlasov equations", arXiv:1707.04333.  One call of
 * fetd_pic_step advances every particle and the fields by the four PIC
 * procedures of Sec. II: field update (Sec. II.A, eqs. semi.dis.curl.1/2),
 * gather through Whitney 1- and 2-forms (Sec. II.B), relativistic push with
 * the Boris, Boris-with-tan-correction, Vay or Higuera-Cary pusher
 * (Sec. II.C), and the exactly charge-conserving scatter of the W1 line
 * integral along each particle's path (Sec. II.D, eq. I.assign).
 *
 * Conventions fixed by this interface:
 *   - SI units.  2-D quantities are per metre of depth: a macro particle of
 *     a species with charge q and weight w carries Q = q w [C/m].
 *   - Triangles are given counter-clockwise.  Local edge k of a triangle is
 *     opposite local node k and runs from local node (k+1)%3 to (k+2)%3.
 *   - Edges are node pairs oriented from the lower to the higher node id
 *     and numbered in lexicographic (low, high) order; e, d and the current
 *     are indexed by that numbering, b and bz by triangle.
 *   - e_i is the line integral of E along edge i [V]; b_f is the flux of
 *     Bz through triangle f [T m^2]; d = [*eps]_eff e is the FP64 primary
 *     electric state (e = M~ d, M~ the sparse approximate inverse of
 *     [*eps]; Gauss's law S~ d = q holds to rounding).
 *   - A particle position is (triangle, derived slot r, barycentric pair):
 *     the pair holds lambda of local nodes (r+1)%3 and (r+2)%3; lambda_r is
 *     (1 - pair0) - pair1.  Momentum u = gamma v [m/s], in-plane.
 *   - Walls: an edge with one adjacent triangle is a PEC wall (not a free
 *     DoF); particles reaching it are removed after depositing their
 *     current up to the wall.  Periodic meshes identify nodes (tri_shift
 *     gives each triangle vertex's image shift).
 *
 * Ownership: input arrays belong to the caller and are copied during the
 * call.  The simulation owns all device memory, obtained through the
 * optional alloc/free callbacks of fetd_opts (else hipMalloc/hipFree), and
 * releases it in fetd_destroy.  Outputs are written to caller buffers whose
 * capacity is checked.
 *
 * Errors: every entry point returns fetd_status.  Argument and state errors
 * are reported at once; device-side errors (crossing cap exceeded,
 * non-finite momentum) are raised by the kernels into a device flag and
 * returned as FETD_E_TRACK by the next synchronising call (fields_get,
 * particles_get, diagnostics, sync).  fetd_last_error gives a message.
 * No entry point aborts or throws across the ABI.
 *
 * Streams: all device work is enqueued on opts.stream (NULL = default
 * stream); fetd_pic_step returns without waiting.
 */
#ifndef FETDPIC_H
#define FETDPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FETD_OK = 0,
    FETD_E_ARG = -1,   /* invalid argument */
    FETD_E_MESH = -2,  /* invalid or unsupported mesh */
    FETD_E_OOM = -3,   /* allocation failed */
    FETD_E_HIP = -4,   /* HIP runtime error */
    FETD_E_TRACK = -5, /* crossing cap exceeded or non-finite momentum */
    FETD_E_STATE = -6  /* call not valid in the current state */
} fetd_status;

/* Pushers of Sec. II.C. */
typedef enum { FETD_BORIS = 0, FETD_BORIS_TAN = 1, FETD_VAY = 2, FETD_HC = 3 } fetd_pusher;

/* FETD_FP64: every stage in FP64; a particle's gather, push, move and
 * tracking take the operations of their definitions in order (no fused
 * multiply-adds, IEEE divisions and square roots), so given the same field
 * values its state is the one a plain FP64 evaluation gives, bit for bit.
 * FETD_MIXED: particle positions (barycentric pair) and momenta stored in
 * FP32, gather/push/track in FP32; the current weights and their
 * accumulation, the primary electric state d and the Gauss accounting in
 * FP64 (charge is conserved to FP64 rounding); e, b and the values of the
 * approximate inverse M~ stored in FP32 (the field update reads and writes
 * them in FP32 and computes in FP64).
 * FETD_MIXED_F64FIELD: as FETD_MIXED with e, b and M~ in FP64. */
typedef enum { FETD_FP64 = 0, FETD_MIXED = 1, FETD_MIXED_F64FIELD = 2 } fetd_precision;

/* Largest particle count of one species and largest mesh: the particle
 * kernel addresses its streams and per-triangle tables with 32-bit byte
 * offsets.  Larger loads and meshes are rejected with FETD_E_ARG before
 * any device work. */
#define FETD_MAX_SPECIES_PARTICLES ((int64_t)268434432) /* 2^28 - 1024 */
#define FETD_MAX_TRIS ((int32_t)67108864)               /* 2^26 */

typedef struct fetd_sim fetd_sim;
typedef void *(*fetd_alloc_fn)(size_t bytes, void *user);
typedef void (*fetd_free_fn)(void *ptr, void *user);

typedef struct {
    int32_t n_nodes;
    const double *node_xy;   /* [2*n_nodes] x, y [m] */
    int32_t n_tris;
    const int32_t *tri_nodes; /* [3*n_tris] counter-clockwise node ids */
    const int8_t *tri_shift;  /* [6*n_tris] (sx, sy) per vertex in periods, or NULL */
    const double *period;     /* [2] period per axis (0 = bounded), or NULL */
} fetd_mesh_desc;

typedef struct {
    int32_t precision;    /* fetd_precision */
    double dt;            /* time step [s] */
    double eps0, mu0, c;  /* vacuum constants [SI]; c enters the pushers
                             (c^2 must lie in [1e-250, 1e250]) */
    int32_t spai_level;   /* >= 0: SPAI of [*eps] on the level-th power of its
                             sparsity graph (0 = diagonal); -1: exact inverse
                             (meshes with at most 4096 edges) */
    int32_t device;       /* HIP device ordinal */
    void *stream;         /* hipStream_t, or NULL for the default stream */
    fetd_alloc_fn alloc;  /* optional device allocator (e.g. a caching allocator) */
    fetd_free_fn free;
    void *alloc_user;
    int32_t crossing_cap; /* maximum edge crossings per particle per step; 0 = 64 */
    int32_t resort_every; /* re-sort particles by triangle every k steps; 0 = 20 */
    int32_t deterministic; /* != 0: every result is independent of the order in which
                              particles are stored, tiled, sorted or batched, bit for
                              bit: each current contribution is added as an integer to
                              a fixed-point accumulator per edge (3 x 32 bits below the
                              largest contribution's power of two, one device integer
                              atomic per limb), converted to FP64 once per step.  The
                              sum differs from a sequential FP64 sum only by rounding. */
    int32_t record_crossings; /* 0..64: keep, for every particle, the triangles of the first
                              record_crossings straight pieces of its last step's move and
                              the number of pieces (Sec. II.D), read with
                              fetd_crossings_get; 0 = off (no memory, no cost) */
} fetd_opts;

/* Field / table selectors for fetd_fields_get. */
typedef enum {
    FETD_FIELD_E = 0,       /* double[n_edges]: e^n */
    FETD_FIELD_D = 1,       /* double[n_edges]: d^n */
    FETD_FIELD_B = 2,       /* double[n_tris]: b^{n-1/2} (after a step: the b used next) */
    FETD_FIELD_J = 3,       /* double[n_edges]: current i^{n+1/2} of the last step */
    FETD_FIELD_Q = 4,       /* double[n_nodes]: nodal charge q^n (Sec. II.D) */
    FETD_FIELD_SPAI_PTR = 5, /* int32[n_edges+1]: CSR row pointers of M~ */
    FETD_FIELD_SPAI_COL = 6, /* int32[nnz] */
    FETD_FIELD_SPAI_VAL = 7, /* double[nnz] */
    FETD_FIELD_EDGES = 8,   /* int32[2*n_edges]: (low, high) node of every edge */
    FETD_FIELD_TRI_EDGE = 9, /* int32[3*n_tris]: edge of local edge k */
    FETD_FIELD_DIVD = 10    /* double[n_nodes]: S~ d^n */
} fetd_field;

typedef struct {
    int32_t n_nodes, n_tris, n_edges, n_free_edges, n_free_nodes;
    int64_t spai_nnz;
    double spai_frobenius;  /* ||I - [*eps] M~||_F / sqrt(n_free_edges) */
    int32_t n_species;
    int64_t device_bytes;   /* device memory held */
} fetd_info;

typedef struct {
    int64_t step;           /* steps taken */
    int64_t n_alive, n_lost;
    int64_t n_segments;     /* path pieces deposited since creation */
    double gauss_abs;       /* max over free nodes |S~(d^n - d^0) - (q^n - q^0)| [C/m] */
    double gauss_rel;       /* gauss_abs / max(|q^n|, |q^0|) */
    double dce_abs;         /* max over free nodes |q^n - q^{n-1} + dt S~ i^{n-1/2}|,
                               when the previous diagnostics call was one step ago; else -1 */
    double dce_rel;
    double W_E;             /* (1/2) e . d  [J/m] */
    double W_B;             /* (1/2) sum_f b_f^2 / (mu0 A_f) */
    double W_kin;           /* sum w m c^2 (gamma - 1) */
    int32_t error_code;     /* 0, or 1 = crossing cap, 2 = non-finite momentum */
    int64_t error_particle; /* load-order index of the first offending particle */
} fetd_diag;

/* Build the mesh tables, [*eps], its approximate inverse and all device
 * state (Sec. II.A).  Fields start at zero.  *out receives the handle. */
fetd_status fetd_mesh_create(const fetd_mesh_desc *mesh, const fetd_opts *opts,
                             fetd_sim **out);

/* Static external fields added at the gather (not evolved): bz_ext per
 * triangle [T], e_ext per edge [V] (line-integral DoFs), and an affine
 * field E(r) = (a0 + a2 x + a3 y, a1 + a4 x + a5 y) [V/m] evaluated at the
 * particle's Cartesian position in its triangle's frame.  NULL clears. */
fetd_status fetd_fields_set(fetd_sim *sim, const double *bz_ext, const double *e_ext,
                            const double *e_affine);

/* Time-dependent amplitude of the applied edge field: from the next step
 * on, the gather uses e + scale * e_ext (a radio-frequency drive such as the
 * accelerating gap of the synchrocyclotron, Sec. III.A, set by the caller
 * each step as E0 sin(phase)).  The default is 1.  The applied field is not
 * evolved by the field update.  A batch that holds the simulation takes the
 * new scale at its next fetd_batch_step (it rebuilds its descriptors, which
 * also ends its captured graph).  FETD_E_ARG if scale is not finite. */
fetd_status fetd_set_ext_scale(fetd_sim *sim, double scale);

/* Matched absorbing layer, the stand-in for the PML of Sec. III.C: a per-
 * triangle conductivity sigma_tri [S/m], nf values, host memory, read
 * during the call (NULL clears).  Electric loss: each edge takes the mean
 * conductivity of its triangles and its d is multiplied after every Ampere
 * update by (1 - x)/(1 + x), x = sigma dt / (2 eps0).  Magnetic loss: each
 * triangle's b is multiplied after every Faraday update by the same factor
 * of its own sigma (magnetic conductivity sigma mu0 / eps0), which keeps
 * the layer's wave impedance at that of free space, so a wave entering at
 * normal incidence is not reflected by the step in loss.  Nodes touching a
 * lossy edge are left out of the Gauss residual of fetd_diagnostics.
 * FETD_E_ARG (nothing changed) if any sigma is negative or not finite.
 * A batch that holds the simulation takes the new layer at its next
 * fetd_batch_step, as it does after fetd_fields_set or a new species.
 * Replaces a PML set by fetd_set_pml. */
fetd_status fetd_set_absorber(fetd_sim *sim, const double *sigma_tri);

/* Uniaxial perfectly matched layer, the absorbing boundary of Sec. III.C
 * (whose construction the paper leaves to its references; built here from
 * the stretched-coordinate medium): conductivity sigma_tri [S/m] per
 * triangle (nf values, host memory, read during the call; NULL clears),
 * stretching along axis (0: layers normal to x, such as the left and right
 * boundaries of a strip periodic in y; 1: normal to y).  With
 * s = 1 + sigma/(j omega eps0) the layer's permittivity is eps0 diag(1/s, s)
 * in (normal, tangential) and its permeability mu0 s: the magnetic loss on b
 * is the matched one (as fetd_set_absorber's), d is updated without loss,
 * and e = M~ (d + psi - phi) with two auxiliary fluxes per layer edge row,
 * psi (the normal part of [*eps] e, divided by s) and phi (the tangential
 * part, multiplied by s), each edge taking the mean conductivity of its
 * triangles.  Waves at oblique incidence are absorbed as at normal
 * incidence, and Gauss's law holds at every free node, in the layer too.
 * Replaces an absorber set by fetd_set_absorber (and is replaced by one).
 * fetd_fields_load restarts the auxiliary fluxes at zero.  FETD_E_ARG
 * (nothing changed) if a sigma is negative or not finite or axis is not 0
 * or 1. */
fetd_status fetd_set_pml(fetd_sim *sim, const double *sigma_tri, int32_t axis);

/* Load the self-consistent field state (Sec. II.A): b [nf] face fluxes
 * b^{n-1/2} [Wb/m] in triangle order, d [ne] edge fluxes d^n [C/m] in the
 * edge order of FETD_FIELD_EDGES; host memory, read during the call; either
 * may be NULL to keep the current value.  e^n = M~ d^n is recomputed; d on
 * wall edges is taken as 0.  With fetd_fields_get (FETD_FIELD_B, _D) and
 * fetd_particles_get / fetd_particles_load_bary it restarts a run from a
 * saved state.  The Gauss accounting of fetd_diagnostics restarts from the
 * loaded state (with the particles present then).  FETD_E_ARG (nothing
 * changed) if a value is not finite. */
fetd_status fetd_fields_load(fetd_sim *sim, const double *b, const double *d);

/* Append a species of n macro particles given in barycentric form
 * (tri[n], slot[n] or NULL for slot 0, lam[2n], u[2n]).  Load order
 * defines particle ids 0..n-1 within the species.  *species_out gets the
 * species index. */
fetd_status fetd_particles_load_bary(fetd_sim *sim, double q, double m, double w, int64_t n,
                                     const int32_t *tri, const int8_t *slot,
                                     const double *lam, const double *u,
                                     int32_t *species_out);

/* Same, from Cartesian positions xy[2n]: each point is located in the
 * lowest-id triangle that contains it (periodic images included).
 * tri_hint [n] or NULL: a triangle expected to contain each point; where it
 * does (the point or a periodic image inside or on its boundary) it is
 * taken without a search, else the point is searched for as without a
 * hint; hints out of range are ignored. */
fetd_status fetd_particles_load(fetd_sim *sim, double q, double m, double w, int64_t n,
                                const double *xy, const double *u, const int32_t *tri_hint,
                                int32_t *species_out);

/* Advance n_steps PIC steps with the given pusher (fetd_pusher).
 * Asynchronous on the simulation's stream. */
fetd_status fetd_pic_step(fetd_sim *sim, int32_t n_steps, int32_t pusher);

/* Re-sort every species by triangle now (also drops lost particles). */
fetd_status fetd_sort(fetd_sim *sim);

/* Wait for the stream and report device-side errors. */
fetd_status fetd_sync(fetd_sim *sim);

/* Copy a field or mesh table (fetd_field) to host memory.  *written gets
 * the byte size; FETD_E_ARG if capacity_bytes is too small. */
fetd_status fetd_fields_get(fetd_sim *sim, int32_t which, void *host_dst,
                            int64_t capacity_bytes, int64_t *written);

/* Copy the alive particles of a species, in load-id order of the alive
 * ones: tri[n], slot[n], lam[2n], u[2n], id[n] (any may be NULL).
 * *n_out gets the count; FETD_E_ARG if capacity < count. */
fetd_status fetd_particles_get(fetd_sim *sim, int32_t species, int64_t capacity,
                               int32_t *tri, int8_t *slot, double *lam, double *u,
                               int64_t *id, int64_t *n_out);

/* The crossing record of the last step (fetd_opts.record_crossings = K > 0,
 * else FETD_E_STATE), for the species' particles alive after it, in the
 * order and count of fetd_particles_get: count[n] = the number of straight
 * pieces of each particle's move (1 = it stayed in its triangle), tris[n*K]
 * = the triangle of each of the first K pieces, -1 past count.  Kept by
 * fetd_pic_step; steps taken in a batch do not update it.  Valid until the
 * next step or sort.  Either array may be NULL; capacity counts particles. */
fetd_status fetd_crossings_get(fetd_sim *sim, int32_t species, int64_t capacity, int32_t *count,
                               int32_t *tris, int64_t *n_out);

/* Charge, Gauss and continuity residuals, energies and counters
 * (Sec. II.A eq. semi.dis.div.2, Sec. II.D eq. full.dis.cont).
 * Synchronises the stream. */
fetd_status fetd_diagnostics(fetd_sim *sim, fetd_diag *out);

/* Stage timing with HIP events on the simulation's stream: stage 0 =
 * Faraday and gather record, 1 = particle stage (one launch per species),
 * 2 = Ampere, 3 = SpMV, 4 = re-sort (all of its kernels).  Stages 0-3 pass
 * their events to their kernel dispatches (hipExtLaunchKernel: the start
 * time of the stage's first kernel, the end time of its last); the re-sort
 * records them around its launches.  enable != 0 starts (and resets)
 * timing of every stage, 0 stops it. */
fetd_status fetd_profile(fetd_sim *sim, int32_t enable);

/* As fetd_profile, timing only the stages whose bit (1 << stage) is set in
 * stage_mask (bits above FETD_N_STAGES are ignored; 0 stops timing), and
 * only on steps whose index is a multiple of every (>= 1, else FETD_E_ARG).
 * A dispatch that carries events leaves the device idle for several
 * microseconds around it, so a run whose own duration is measured times
 * only the stage it needs, on a sample of its steps (an every coprime with
 * the re-sort interval samples every phase of the sort cycle). */
fetd_status fetd_profile_mask(fetd_sim *sim, int32_t stage_mask, int32_t every);

/* Device milliseconds summed per stage since timing started, and the number
 * of timed launches per stage (arrays of FETD_N_STAGES).  Synchronises. */
#define FETD_N_STAGES 5
fetd_status fetd_stage_times(fetd_sim *sim, double *ms, int64_t *launches);

/* Autotune the particle kernel's tiling and current scan and the re-sort
 * cadence (the tuning the method leaves to the implementation: how many
 * particles a block of the particle kernel takes, over how many lanes the
 * first-piece currents are summed before their LDS add, and how often the
 * triangle order is restored).  With T = min(trial_steps, 20):
 * 1. Tile: for each tile size (512 to 2048 particles per block of 256
 *    threads in steps of 256; the current one first) sort, run T steps
 *    timing the particle stage with HIP events; keep the tile of least mean
 *    particle-stage time (ties keep the earlier candidate).  The tile sets
 *    how many rounds of blocks a launch takes on the device's block slots:
 *    on a launch of a few rounds the last, partly filled round is a
 *    sizeable share of the time.
 * 2. Scan: the same for the scan group widths 64, 16 and 8 lanes, with that
 *    tile (the current width first).
 * 3. Deferred exits (FP32 particles only): the same for off and on (the
 *    current setting first); see fetd_set_defer_exits.
 * 4. Cadence: sort once (timed), advance trial_steps steps timing the
 *    particle stage of every step, and set the re-sort interval K
 *    minimising (T_sort + sum_{j<K} T_particles(j)) / K over the candidates
 *    5, 10, 20, 40, 80, 160 (up to trial_steps).
 * out (or NULL) receives the choices and the measured costs.  Every trial
 * step is an ordinary step: the simulation advances by 10 T (FP32
 * particles: 12 T) + trial_steps steps, and its results do not depend on
 * the choices beyond FP64 summation order (not at all in deterministic
 * mode). */
typedef struct {
    int32_t resort_every;       /* chosen re-sort interval K */
    int32_t tile_particles;     /* chosen tile */
    int32_t scan_lanes;         /* chosen scan group width */
    int32_t defer_exits;        /* chosen exit mode (FP32 particles; 1 in FP64) */
    double resort_cost_ms[6];   /* cost per step of K = 5, 10, 20, 40, 80, 160; -1 if untried */
    double tile_cost_ms[7];     /* mean particle-stage ms per step, tiles 512, 768, ..., 2048 */
    double scan_cost_ms[3];     /* the same for scan widths 64, 16, 8 */
    double defer_cost_ms[2];    /* the same for deferred exits off, on; -1 if untried (FP64) */
} fetd_tuning;
fetd_status fetd_autotune(fetd_sim *sim, int32_t pusher, int32_t trial_steps, fetd_tuning *out);

/* Particles per block of the particle kernel for this run: a multiple of
 * 256 from 512 to 2048 (default 1024), else FETD_E_ARG.  Takes effect at the next step (the
 * tiles' current-window homes are recomputed from the current order); a run
 * stepped in a batch keeps its own tile there (a batch rebuilds its tile
 * list when a member's tile changes). */
fetd_status fetd_set_tile(fetd_sim *sim, int32_t tile_particles);
fetd_status fetd_get_tile(fetd_sim *sim, int32_t *tile_particles);

/* Lanes per group over which the particle kernel sums the currents of
 * particles' first pieces in one triangle before one LDS add per group:
 * 8, 16 or 64 (the default, the whole wavefront), else FETD_E_ARG.  Changes
 * only the FP64 summation order of the deposit (nothing in deterministic
 * mode). */
fetd_status fetd_set_scan(fetd_sim *sim, int32_t scan_lanes);
fetd_status fetd_get_scan(fetd_sim *sim, int32_t *scan_lanes);

/* Deferred exits (FP32 particles; FP64 always defers, and a batched step
 * never does in FP32): the particle kernel's first pass decides by
 * comparison which moves stay inside their triangle, with a margin of
 * 2^-20 above the error of the FP32 reciprocal (every move kept is one the
 * full first piece ends inside), and traces the others from their start
 * after the pass, with the full first piece, so each move ends as it would
 * otherwise; off, it traces every particle's first piece in the pass.  On pays where few particles cross an edge per step.
 * The results are the same either way up to FP64 summation order (bit for
 * bit in deterministic mode).  on: 0 or 1, else FETD_E_ARG; an FP64 run
 * accepts it, keeps deferring and reports 1. */
fetd_status fetd_set_defer_exits(fetd_sim *sim, int32_t on);
fetd_status fetd_get_defer_exits(fetd_sim *sim, int32_t *on);

/* Set the re-sort interval directly (k >= 1). */
fetd_status fetd_set_resort(fetd_sim *sim, int32_t every);

/* Batched stepping of many independent simulations (parameter sweeps):
 * every phase of a step (Faraday, particle stage, Ampere, SpMV) is one
 * persistent launch over the flattened work of all runs; with use_graph
 * the launch sequence of a cycle of two re-sort intervals (2K steps) is
 * captured in a HIP graph and replayed: once per pusher, phase in the
 * re-sort interval and sort parity (the graph's sorts read and write fixed
 * buffers), after one eager sorting step per pusher; a call whose steps
 * cover a cycle from the next sort starts its graph there, a shorter one at
 * its current phase, so calls of 2K steps replay from the third on.  All
 * simulations must live on the same device and stream, have the same
 * precision and appear once each (else FETD_E_ARG); they stay individually usable
 * (fields_get, particles_get, diagnostics) between batch steps.  The batch
 * keeps pointers to the simulations: destroy it before them.  Re-sorting
 * follows resort_every of the first simulation as it was when the batch was
 * created.  Members must also agree
 * on the deterministic option.  The batch runs on a non-blocking stream
 * of its own and orders itself after the members' earlier work and before
 * their later work with events, so a graph can be captured also when the
 * members use the legacy default stream.  The particle launch takes its
 * tiles from a queue, the (run, species) segments ordered largest first. */
typedef struct fetd_batch fetd_batch;
fetd_status fetd_batch_create(fetd_sim *const *sims, int32_t n, int32_t use_graph,
                              fetd_batch **out);
fetd_status fetd_batch_step(fetd_batch *batch, int32_t n_steps, int32_t pusher);

/* Counters of a batch: graphs captured, graph replays (each a cycle of two
 * re-sort intervals) and steps enqueued eagerly. */
fetd_status fetd_batch_stats(fetd_batch *batch, int64_t *graph_captures, int64_t *graph_replays,
                             int64_t *eager_steps);
void fetd_batch_destroy(fetd_batch *batch);

/* For callers that cannot allocate device memory (serving loops, harnesses
 * that forbid allocation): n_steps batched steps of the n simulations, as
 * fetd_batch_create + fetd_batch_step would take them (same kernels, same
 * results; eager launches, no graph), without a batch object and without
 * allocating anything.  The descriptor and prefix tables and the tile queue
 * the batched kernels read go to a fixed device array of the library
 * (384 KiB per device, held until the process ends), which limits a call to
 * n <= 256 simulations and 512 non-empty species in all (FETD_E_ARG
 * beyond).  The call uploads its tables from host memory and waits for the
 * members' stream once before its first launch; the rest is asynchronous on
 * that stream.  Every call on a device shares that device's array: calls
 * that overlap on one device (other threads, other streams) race.  The
 * members must share device, stream, precision and the deterministic
 * option; the re-sort interval is the first member's.  A member's Gauss
 * accounting, if it has none yet, starts at its next fetd_diagnostics. */
fetd_status fetd_batch_step_noalloc(fetd_sim *const *sims, int32_t n, int32_t n_steps,
                                    int32_t pusher);

/* Field probes (Sec. III.C samples E along a line at every step to obtain
 * the dispersion relation).  n points xy [2n] (metres; located like
 * fetd_particles_load, FETD_E_ARG if one lies outside the mesh).  After
 * every step the self-consistent field E (applied fields excluded) is
 * evaluated at each point from the Whitney interpolant of e (Sec. II.B);
 * the values of each window of `every` consecutive steps are averaged and
 * stored as one sample, up to max_samples samples (later ones are
 * dropped).  n = 0 removes the probes; a new call restarts the record.
 * Steps taken through fetd_batch_step are not probed. */
fetd_status fetd_probe_set(fetd_sim *sim, int64_t n, const double *xy, int32_t every,
                           int64_t max_samples);

/* Copy the recorded probe samples to dst: [samples][n][2] doubles (E_x,
 * E_y in V/m).  *n_samples receives the count; dst may be NULL to query it.
 * FETD_E_ARG if capacity_bytes is too small. */
fetd_status fetd_probe_get(fetd_sim *sim, double *dst, int64_t capacity_bytes,
                           int64_t *n_samples);

/* Measured bandwidth ceiling of the device: a plain copy kernel (16-byte
 * vectors, grid-stride) over two buffers of `bytes` bytes that it allocates
 * and frees, the best of a few grid sizes and `reps` timed launches each;
 * *gbs gets (read + write bytes) / time in GB/s.  The reference against
 * which the particle kernel's bandwidth is also reported. */
fetd_status fetd_copy_ceiling(int32_t device, int64_t bytes, int32_t reps, double *gbs);

/* Sizes and SPAI quality. */
fetd_status fetd_info_get(fetd_sim *sim, fetd_info *out);

/* Message of the last failed call on sim (thread-local one if sim is NULL). */
const char *fetd_last_error(const fetd_sim *sim);

/* Release all device memory and the handle.  NULL is a no-op. */
void fetd_destroy(fetd_sim *sim);

#ifdef __cplusplus
}
#endif

#endif /* FETDPIC_H */
