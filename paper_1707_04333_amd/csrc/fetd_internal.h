// Internal declarations shared by the host runtime and the HIP kernels of
// the FETD-PIC library.  Not part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fetd {

constexpr uint32_t kLost = 0xFFFFFFFFu;   // key of a removed particle
constexpr uint32_t kTriMask = 0x3FFFFFFFu; // triangle id bits of a key
constexpr int kBlock = 256;                // threads per block of the particle kernels
#ifndef FETD_PPT
#define FETD_PPT 4
#endif
constexpr int kPPT = FETD_PPT;             // default particles per thread of the particle kernel
// Particles per thread a run may use (its tile is ppt * kBlock particles,
// 512 to 2048 in steps of 256, a run-time value of the step arguments);
// per-tile slots are sized for the smallest.
constexpr int kNumPPT = 7;
constexpr int kPPTChoices[kNumPPT] = {2, 3, 4, 5, 6, 7, 8};
constexpr int kMinPPT = 2;
inline bool valid_ppt(int p) { return p >= kMinPPT && p <= 8; }
// Lanes per group of the first-piece current scan (a run-time value).
constexpr int kScanChoices[3] = {64, 16, 8};
inline bool valid_scan(int w) { return w == 8 || w == 16 || w == 64; }
constexpr int kSlice = 64;                 // rows per SELL slice of the SpMV

// Per-triangle tables (device).
//   tri_edge[f] = {edge of local edge 0, 1, 2, sign bits: bit k set when
//                  local edge k runs against the global orientation}
//   tri_nbr[f]  = {neighbour across local edge 0, 1, 2 (-1 = wall),
//                  local index of the shared edge in the neighbour, 2 bits each}
struct MeshView {
    const int4 *tri_edge;
    const int4 *tri_nbr;
    const double *grad64;  // [nf*6]: (gx, gy) of local node 0, 1, 2
    const float *grad32;   // [nf*8]: same in FP32, padded to 32 B
    const double *vxy64;   // [nf*6]: image-consistent vertex coordinates
    const float *vxy32;    // [nf*8]
    // Edges are numbered on the device in order of first appearance along
    // the triangle order; tri_ebase[f] = number of edges first met before
    // triangle f (the edges of f and of its near successors lie at or above).
    const uint32_t *tri_ebase;
};

// LDS current window of a particle tile: kWin consecutive device edge ids
// starting at the edges of the triangle kWinBack before the tile's home
// triangle (the triangle of its first particle at the last sort).
constexpr int kWin = 2048;
constexpr uint32_t kWinBack = 512;

// Arguments of one particle-stage launch (one species).
struct StepArgs {
    int64_t n;
    uint32_t *key;
    void *lam;        // double2 or float2 [n]: barycentric pair
    void *u;          // double2 or float2 [n]: momentum u = gamma v
    const void *rec;  // per-triangle field record, 32 B: FP32 V0, V1, V2 (E = sum l_n V_n), Bz,
                      // pad; FP64 the signed edge DoFs s_k e_k and Bz
    double *cur;      // FP64 current accumulator [ne]
    unsigned long long *fx;  // deterministic mode: fixed-point current limbs [3 ne], else null
    double fx_scale;  // 2^(96 - E) with every contribution below 2^E in magnitude
    double qdt;       // Q / dt of the species
    double alpha;     // q dt / (2 m)
    double dt;
    double c;
    double c2;        // c * c
    double inv_c2;    // 1 / (c * c)
    int cap;          // crossing cap
    int has_affine;
    double aff[6];
    unsigned long long *counters;  // [2] error flags, [3] first bad id (rarely written)
    unsigned long long *block_counts;  // [2 * tiles]: per-tile running sums (segments, lost)
    const uint32_t *tile_home;     // [tiles]: home triangle of each tile (set by the sort)
    const int32_t *pid;            // load ids (for error reports)
    int ppt;                       // particles per thread: a tile is ppt * kBlock particles
    int scan;                      // lanes per group of the first-piece current scan (8, 16, 64)
    int defer;                     // FP32: deferred exits (FP64 always defers; batched: never)
    int32_t *xcount;               // crossing record, or null: pieces of each particle's move
    int32_t *xtris;                // [n * xcap]: the triangle of each of the first xcap pieces
    int xcap;
};

// One (run, species) segment of a batched particle launch.
struct SegDesc {
    MeshView m;
    StepArgs a;
};

// Field stages of one run (passed by value to the single-run kernels, as
// an array to the batched ones).  e, b, h, the values of M~ and e_out are
// FP64, or FP32 when field32 is set; d and the currents are FP64.
struct FieldDesc {
    int nf, ne;
    int rec_fp32;     // field record for FP32 particles (else the FP64 record)
    int field32;
    const int4 *tri_edge;
    const void *e;
    const double *e_ext;
    double e_scale;   // multiplier of e_ext
    void *b;
    const double *damp_b;  // magnetic loss per triangle (absorbing layer) or null
    void *h;               // b / (mu0 A)
    const double *mu_area;   // mu0 A_f
    const double *two_area;  // 2 A_f
    const double *bz_ext;
    const double *grad64;
    void *rec;
    double dt;
    const int4 *edge_face;
    double *cur;
    double *cur_last;
    double *d;
    const double *damp;
    unsigned long long *fx;  // deterministic mode: fixed-point current limbs, else null
    double fx_unscale;       // 2^(E - 96)
    // uniaxial PML (pml_n rows, else 0): device edge id and kappa = sigma/eps0
    // per row, the rows of the normal (pn) and tangential (pt) parts of
    // [*eps] (CSR, device edge columns), the auxiliary fluxes psi, phi per
    // row, and pml_x = psi - phi per edge (zero off the layer; null without
    // a PML), which the SpMV adds to d
    int pml_n;
    const int32_t *pml_rows;
    const double *pml_kappa;
    const int32_t *pn_ptr, *pn_col;
    const double *pn_val;
    const int32_t *pt_ptr, *pt_col;
    const double *pt_val;
    double *pml_psi, *pml_phi, *pml_x;
    const int32_t *sl_ptr;
    const int32_t *sl_w;
    const int32_t *sl_col;
    const void *sl_val;
    void *e_out;
};

// Host-callable launchers (fetd_kernels.hip).
hipError_t launch_faraday(hipStream_t s, const FieldDesc &d);
hipError_t launch_ampere(hipStream_t s, const FieldDesc &d);
hipError_t launch_spmv(hipStream_t s, const FieldDesc &d);
// PML auxiliary fluxes from the current e (before the SpMV of the step).
hipError_t launch_pml_aux(hipStream_t s, const FieldDesc &d);

// Particle stage (fetd_particles.hip, one object per precision).  A
// deterministic launch is selected by a.fx != null (batched: det); a.ppt
// is one of kPPTChoices.
hipError_t launch_particles_f32(hipStream_t s, const MeshView &m, const StepArgs &a, int pusher);
hipError_t launch_particles_f64(hipStream_t s, const MeshView &m, const StepArgs &a, int pusher);
// Batched: queue = [next tile, blocks done], zero before the first launch;
// the kernel's last block leaves it at zero again.
hipError_t launch_particles_batched_f32(hipStream_t s, const SegDesc *segs, const uint32_t *prefix,
                                        int nseg, uint32_t total_tiles, uint32_t *queue,
                                        int pusher, bool det);
hipError_t launch_particles_batched_f64(hipStream_t s, const SegDesc *segs, const uint32_t *prefix,
                                        int nseg, uint32_t total_tiles, uint32_t *queue,
                                        int pusher, bool det);
inline hipError_t launch_particles(hipStream_t s, const MeshView &m, const StepArgs &a, int pusher,
                                   bool fp32)
{
    return fp32 ? launch_particles_f32(s, m, a, pusher) : launch_particles_f64(s, m, a, pusher);
}
inline hipError_t launch_particles_batched(hipStream_t s, const SegDesc *segs,
                                           const uint32_t *prefix, int nseg, uint32_t total_tiles,
                                           uint32_t *queue, int pusher, bool fp32, bool det)
{
    return fp32 ? launch_particles_batched_f32(s, segs, prefix, nseg, total_tiles, queue, pusher,
                                               det)
                : launch_particles_batched_f64(s, segs, prefix, nseg, total_tiles, queue, pusher,
                                               det);
}

// Largest species and mesh the 32-bit byte offsets of the particle kernel
// address (16-byte FP64 particle records, 48-byte triangle tables).
constexpr int64_t kMaxSpeciesParticles = (int64_t(1) << 28) - 1024;
constexpr int64_t kMaxTris = int64_t(1) << 26;

// Counting sort of one species segment by triangle (drops lost particles).
// counts/offsets need nf+1 ints, block_sums a few thousand.
struct SortArgs {
    int64_t n;
    int nf;
    const uint32_t *key_in;
    const void *lam_in;
    const void *u_in;
    const int32_t *pid_in;
    uint32_t *key_out;
    void *lam_out;
    void *u_out;
    int32_t *pid_out;
    int32_t *counts;   // [nf + 1]
    int32_t *offsets;  // [nf + 1]
    int32_t *block_sums;
    int elem_bytes;    // 8 (float2) or 16 (double2)
    uint32_t *tile_home;  // [tiles of n]: triangle of each tile's first particle after the sort
    int64_t tile;         // particles per tile of the particle kernel
};
hipError_t launch_sort(hipStream_t s, const SortArgs &a);
// tile_home of n keys in their current order, tiles of `tile` particles.
hipError_t launch_tile_home(hipStream_t s, int64_t n, const uint32_t *key, uint32_t *home,
                            int64_t tile);

// Batched launches over many runs (one launch per phase).
hipError_t launch_faraday_batched(hipStream_t s, const FieldDesc *d, const uint32_t *prefix,
                                  int nrun, uint32_t total_blocks);
hipError_t launch_ampere_batched(hipStream_t s, const FieldDesc *d, const uint32_t *prefix,
                                 int nrun, uint32_t total_blocks);
hipError_t launch_spmv_batched(hipStream_t s, const FieldDesc *d, const uint32_t *prefix,
                               int nrun, uint32_t total_blocks);
hipError_t launch_fill_u32(hipStream_t s, uint32_t *p, uint32_t v, int64_t n);
// Field probes: accumulate E at n points; when out is non-null write the
// window average there (times inv_window) and restart the sum.
hipError_t launch_probe(hipStream_t s, int n, const int32_t *tri, const double *lam,
                        const int4 *tri_edge, const double *grad64, const void *e, bool field32,
                        double *acc, double *out, double inv_window);

// Copy of n16 16-byte vectors with `blocks` blocks of 256 threads (bandwidth ceiling).
hipError_t launch_copy(hipStream_t s, const void *src, void *dst, int64_t n16, int blocks);

// Diagnostics.
hipError_t launch_charge(hipStream_t s, int64_t n, const uint32_t *key, const void *lam,
                         bool fp32, const int4 *tri_node, double qw, double *q);
hipError_t launch_divd(hipStream_t s, int ne, const int2 *edge_nodes, const double *d,
                       double *out);
hipError_t launch_kinetic(hipStream_t s, int64_t n, const uint32_t *key, const void *u, bool fp32,
                          double inv_c2, double *partial, int n_partial);

}  // namespace fetd
