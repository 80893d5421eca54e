// Internal declarations of the tetrahedral path (host runtime <-> HIP
// kernels).  Not part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fetd3 {

constexpr uint32_t kLost = 0xFFFFFFFFu;    // key of a removed particle
constexpr uint32_t kTetMask = 0x3FFFFFFFu; // tetrahedron bits of a key (slot in bits 30-31)
constexpr int kBlock = 256;

// Per-tetrahedron tables (device):
//   tet_edge[8t + k], k < 6: global edge of local edge k; tet_edge[8t + 6]:
//     bit k set when local edge k runs against its global edge, bits 8-11:
//     bit 8+k set when local face k (local sorted order) is an odd
//     permutation of its global face; tet_edge[8t + 7] unused;
//   tet_face[t] = global faces of local faces 0-3;
//   tet_nbr[t]  = neighbour across local face 0-3 (-1 = wall);
//   tet_map[t]  = byte k for face k: local index in the neighbour of local
//     node (k+1)%4, (k+2)%4, (k+3)%4 (2 bits each) and of the neighbour's
//     node opposite the shared face (bits 6-7);
//   grad[12t]   = grad lambda_0..3 (x, y, z).
struct Mesh3 {
    const int32_t *tet_edge;
    const int4 *tet_face;
    const int4 *tet_nbr;
    const uint32_t *tet_map;
    const double *grad;
    const float *grad32;  // same in FP32 (mixed mode)
    // edges are numbered on the device in order of first appearance along
    // the tetrahedron order; tet_ebase[t] = edges first met before t
    const uint32_t *tet_ebase;
};

// LDS current window of a particle block: kWin3 consecutive device edge
// ids starting kBack3 below the first edge id met at the block's home
// tetrahedron (the tetrahedron of its first particle).
constexpr int kWin3 = 2048;
constexpr int kBack3 = 1024;
// Open-addressing table of the block for edges outside the window.
constexpr int kHashBits3 = 8;
constexpr int kHash3 = 1 << kHashBits3;

// Counting sort: particles per block, and the block's LDS window of
// tetrahedron ids (kSortBins3 ids from kSortBack3 below its first particle's).
constexpr int kSortB3 = 1024;
constexpr int kSortBins3 = 1024;
constexpr int kSortBack3 = 256;

// Per-tetrahedron gather record, 24 doubles: V_0..V_3 with E = sum l_n V_n,
// then U_0..U_3 with B = sum l_n U_n (B at time n from the face average).
constexpr int kRec = 24;

struct Step3 {
    int64_t n;
    int64_t stride;     // component stride of lam and u
    uint32_t *key;
    void *lam;          // [3][stride] stored barycentrics (SoA; double, or float when mixed)
    void *u;            // [3][stride] momenta (SoA; same type)
    const void *rec;    // [24 nt] gather records (same type)
    const double *b_ext;  // [3 nt] or null
    double *cur;        // [ne]
    double qdt, alpha, dt, c, inv_c2;
    int cap;
    unsigned long long *counters;  // [0] pieces, [1] lost, [2] error flags, [3] first bad particle
};

struct Sort3 {
    int64_t n;
    int nt;
    const uint32_t *key_in;
    const void *lam_in, *u_in;
    const int32_t *pid_in;
    uint32_t *key_out;
    void *lam_out, *u_out;
    int elem_bytes;  // 8 (double) or 4 (float) per component
    int32_t *pid_out;
    int64_t stride_in, stride_out;  // component stride of the SoA arrays
    int32_t *counts;      // [nt + 1]
    int32_t *cursor;      // [nt + 1]
    int32_t *chunk_sums;  // [ceil((nt + 1) / 1024)]
    int32_t *perm;        // [n] input index of each output slot
};

// Sliced-ELL sparse matrix: 64-row slices, column-major inside a slice.
struct Sell {
    const int32_t *sptr;  // [slices] first entry of each slice
    const int32_t *sw;    // [slices] width of each slice
    const int32_t *col;
    const double *val;
};

hipError_t launch3_faraday(hipStream_t s, int nf, const int4 *face_edge, const double *e,
                           double *b, double *bavg, double dt);
hipError_t launch3_record(hipStream_t s, int nt, const Mesh3 &m, const double *e,
                          const double *e_ext, const double *bavg, void *rec, bool fp32);
hipError_t launch3_particles(hipStream_t s, const Mesh3 &m, const Step3 &a, int pusher,
                             bool fp32);
hipError_t launch3_hnu(hipStream_t s, int nf, const Sell &m, const double *b, double *h);
hipError_t launch3_ampere(hipStream_t s, int ne, const int32_t *ef_ptr, const int32_t *ef_face,
                          const uint8_t *edge_free, const double *h, double *cur,
                          double *cur_last, double *d, double dt);
hipError_t launch3_spmv(hipStream_t s, int ne, const Sell &m, const uint8_t *edge_free,
                        const double *d, double *e);
hipError_t launch3_sort(hipStream_t s, const Sort3 &a);
hipError_t launch3_charge(hipStream_t s, int64_t n, const uint32_t *key, const void *lam,
                          bool fp32, int64_t stride, const int4 *tet_node, double qw, double *q);
hipError_t launch3_divd(hipStream_t s, int ne, const int2 *edge_nodes, const double *d,
                        double *out);
hipError_t launch3_divb(hipStream_t s, int nt, const int4 *tet_face, const int32_t *fout_bits,
                        const double *b, double *out);

}  // namespace fetd3
