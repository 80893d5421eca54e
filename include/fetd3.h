/*
 * C-ABI of the tetrahedral (three-dimensional) FETD-PIC path: the method of
 * Na, Moon, Omelchenko and Teixeira (arXiv:1707.04333), Sec. II, in the
 * general form its Whitney-form formulation states it: e on edges
 * (Whitney 1-forms), b on faces (Whitney 2-forms), incidence C (faces x
 * edges) and S (cells x faces), Hodge matrices [*eps] on edges and
 * [*mu^-1] on faces, a sparse approximate inverse of [*eps], the four
 * relativistic pushers of Sec. II.C and the charge-conserving scatter of
 * Sec. II.D on the six edges of a tetrahedron.  FP64, or the mixed mode
 * of fetd3_opts.precision.
 *
 * Conventions (pinned by the tests):
 *   - tetrahedra are positively oriented (det[x1-x0, x2-x0, x3-x0] > 0);
 *     local edges are (0,1) (0,2) (0,3) (1,2) (1,3) (2,3); local face k is
 *     opposite local node k;
 *   - a global edge runs from its lower to its higher node id; a global
 *     face is the sorted triple (i<j<l) of node ids with normal
 *     (x_j - x_i) x (x_l - x_i); edges and faces are numbered in
 *     lexicographic order of their node ids; C has +1 on (i,j) and (j,l)
 *     and -1 on (i,l);
 *   - b_f is the flux of B through face f along its normal; e_i the line
 *     integral of E along edge i; d = [*eps] e (the primary state, e is
 *     M~ d with M~ the approximate inverse);
 *   - a particle lives in a tetrahedron with a derived slot r in 0..3 and
 *     the barycentrics of local nodes (r+1)%4, (r+2)%4, (r+3)%4; the fourth
 *     is ((1 - s0) - s1) - s2.  Momenta are u = gamma v [m/s]; the macro
 *     charge of a particle is q w.
 *   - faces with one tetrahedron are perfectly conducting walls: their
 *     edges and nodes carry no degree of freedom (e = d = 0) and particles
 *     that reach them are removed after depositing their current up to the
 *     wall.  Periodic meshes give each tetrahedron vertex an image shift.
 *
 * Every call returns fetd_status (fetdpic.h); inputs are host memory read
 * during the call; outputs are written to caller buffers; the simulation
 * owns its device memory and releases it in fetd3_destroy.  Device-side
 * errors (crossing cap, non-finite momentum) are reported as FETD_E_TRACK
 * by the next synchronising call (fields_get, particles_get, diagnostics,
 * sync).
 */
#ifndef FETD3_H
#define FETD3_H

#include <stdint.h>

#include "fetdpic.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fetd3_sim fetd3_sim;

typedef struct {
    int32_t n_nodes;
    const double *node_xyz;   /* [3 n_nodes] m */
    int32_t n_tets;
    const int32_t *tet_nodes; /* [4 n_tets], positively oriented */
    const int8_t *tet_shift;  /* [12 n_tets] image shift of each vertex, or NULL */
    const double *period;     /* [3] period per axis (0 = none), or NULL */
} fetd3_mesh_desc;

typedef struct {
    double dt, eps0, mu0, c;  /* time step [s] and constants (SI) */
    int32_t spai_level;       /* pattern = level-th power of the graph of [*eps] (1..2) */
    int32_t device;           /* HIP device ordinal */
    void *hip_stream;         /* stream to run on, or NULL for a private one */
    int32_t crossing_cap;     /* faces a particle may cross per step (0 = 64) */
    int32_t resort_every;     /* steps between sorts by tetrahedron (0 = 20) */
    int32_t precision;        /* FETD_FP64, or FETD_MIXED: FP32 particle state, gather, push
                                 and march; FP64 barycentrics in flight, deposit, currents
                                 and field update (charge conservation stays at FP64
                                 rounding: FP32 products are exact in FP64) */
} fetd3_opts;

enum {
    FETD3_FIELD_E = 0,      /* double [n_edges] e^n */
    FETD3_FIELD_D = 1,      /* double [n_edges] d^n */
    FETD3_FIELD_B = 2,      /* double [n_faces] b^{n-1/2} */
    FETD3_FIELD_J = 3,      /* double [n_edges] current i^{n-1/2} of the last step */
    FETD3_FIELD_Q = 4,      /* double [n_nodes] nodal charge q = sum Q lambda */
    FETD3_FIELD_DIVD = 5,   /* double [n_nodes] S~ d (net outflow at each node) */
    FETD3_FIELD_DIVB = 6,   /* double [n_tets] S b (net outward flux of each cell) */
    FETD3_FIELD_EDGES = 7,  /* int32 [2 n_edges] (low, high) node ids */
    FETD3_FIELD_FACES = 8,  /* int32 [3 n_faces] sorted node ids */
    FETD3_FIELD_SPAI_PTR = 9,
    FETD3_FIELD_SPAI_COL = 10,
    FETD3_FIELD_SPAI_VAL = 11
};

typedef struct {
    int64_t step, n_alive, n_lost, n_segments;
    int32_t n_nodes, n_edges, n_faces, n_tets;
    double gauss_rel;   /* max over free nodes |S~(d - d0) - (q - q0)| / max|q| */
    double divb_rel;    /* max |S b| / max |b| */
    double W_E;         /* (1/2) e . d [J] */
    double W_B;         /* (1/2) b . [*mu^-1] b */
    double W_kin;       /* sum w m c^2 (gamma - 1) */
    double spai_frobenius;
    int32_t error_code; /* 0, 1 = crossing cap, 2 = non-finite momentum */
} fetd3_diag;

/* Build topology, incidence, Whitney geometry, [*eps], [*mu^-1] and the
 * SPAI of [*eps] (Sec. II.A), and the device state.  Fields start at 0.
 * FETD_E_MESH for an inverted tetrahedron or a non-manifold mesh. */
fetd_status fetd3_mesh_create(const fetd3_mesh_desc *mesh, const fetd3_opts *opts,
                              fetd3_sim **out);

/* Static applied fields added at the gather: b_ext [3 n_tets] (a constant
 * B per tetrahedron, T) and e_ext [n_edges] (edge line integrals, V).
 * NULL clears. */
fetd_status fetd3_fields_set(fetd3_sim *sim, const double *b_ext, const double *e_ext);

/* Load the field state b^{n-1/2} [n_faces] and d^n [n_edges] (either may be
 * NULL to keep it); e = M~ d is recomputed, d on wall edges is taken as 0,
 * and the Gauss accounting restarts from this state. */
fetd_status fetd3_fields_load(fetd3_sim *sim, const double *b, const double *d);

/* Append a species of n particles (tet[n], slot[n] or NULL for slot 0,
 * lam[3n], u[3n]); *species_out gets its index.  Load order defines the
 * particle ids 0..n-1 of the species; every species is then sorted by
 * tetrahedron (storage order only). */
fetd_status fetd3_particles_load_bary(fetd3_sim *sim, double q, double m, double w, int64_t n,
                                      const int32_t *tet, const int8_t *slot, const double *lam,
                                      const double *u, int32_t *species_out);

/* Advance n_steps steps (Sec. II: Faraday half, gather, push, move and
 * deposit, Ampere half) with the pusher of fetd_pusher.  Asynchronous. */
fetd_status fetd3_pic_step(fetd3_sim *sim, int32_t n_steps, int32_t pusher);

/* Sort every species by tetrahedron now (drops removed particles). */
fetd_status fetd3_sort(fetd3_sim *sim);

/* Wait for the stream; FETD_E_TRACK if a device error was raised. */
fetd_status fetd3_sync(fetd3_sim *sim);

/* Copy one field or table (FETD3_FIELD_*) to dst; *written gets the byte
 * size (dst may be NULL to query it); FETD_E_ARG if capacity_bytes is too
 * small. */
fetd_status fetd3_fields_get(fetd3_sim *sim, int32_t which, void *dst, int64_t capacity_bytes,
                             int64_t *written);

/* Particles of one species still in the mesh, in id order: tet, slot,
 * lam [3n], u [3n], id; *n_out gets the count (arrays may be NULL to query
 * it); FETD_E_ARG if capacity is too small. */
fetd_status fetd3_particles_get(fetd3_sim *sim, int32_t species, int64_t capacity, int32_t *tet,
                                int8_t *slot, double *lam, double *u, int32_t *id,
                                int64_t *n_out);

/* Residuals, energies and counts (synchronises). */
fetd_status fetd3_diagnostics(fetd3_sim *sim, fetd3_diag *out);

/* Per-stage device time with HIP events: enable != 0 starts (and resets)
 * timing of every stage, 0 stops it; fetd3_profile_mask times only the
 * stages whose bit (1 << stage) is set (stages: 0 Faraday + record,
 * 1 particles, 2 Ampere, 3 SpMV, 4 sort), on steps whose index is a
 * multiple of every (>= 1, else FETD_E_ARG).  Stages 0-3 pass their events
 * to their kernel dispatches (hipExtLaunchKernel: start of the first
 * kernel, end of the last); the sort records them around its launches.  A
 * dispatch that carries events leaves the device idle for several
 * microseconds around it.  fetd3_stage_times: ms[5] gets the accumulated
 * milliseconds per stage, *launches the particle launches timed. */
fetd_status fetd3_profile(fetd3_sim *sim, int32_t enable);
fetd_status fetd3_profile_mask(fetd3_sim *sim, int32_t stage_mask, int32_t every);
fetd_status fetd3_stage_times(fetd3_sim *sim, double *ms, int64_t *launches);

/* Message of the last failed call on sim (thread-local one if sim is NULL). */
const char *fetd3_last_error(const fetd3_sim *sim);

/* Release all device memory and the handle.  NULL is a no-op. */
void fetd3_destroy(fetd3_sim *sim);

#ifdef __cplusplus
}
#endif

#endif
