// Host runtime of the tetrahedral FETD-PIC path: mesh topology and Whitney
// geometry, the Hodge matrices [*eps] (edges) and [*mu^-1] (faces), the
// sparse approximate inverse of [*eps], device state and the C-ABI entry
// points declared in include/fetd3.h.
//
// Method: arXiv:1707.04333 (Na, Moon, Omelchenko, Teixeira), Sec. II, in
// the dimension-independent Whitney-form statement of its field update.
#include "fetd3.h"
#include "fetd3_internal.h"
#include "fetd_sparse.h"
#include "stage_events.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace fetd3;
using fetd::Csr;

namespace {

thread_local std::string g_err3;

constexpr int LE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
constexpr int LF[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};

struct Species3 {
    double q = 0, m = 0, w = 0;
    int64_t n_loaded = 0;  // ids 0..n_loaded-1
    int64_t n = 0;         // slots in use
    int64_t offset = 0;    // first slot
};

struct DeviceGuard3 {
    int prev = -1;
    explicit DeviceGuard3(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard3()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

struct fetd3_sim {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    double dt = 0, eps0 = 0, mu0 = 0, c = 0;
    int spai_level = 1, cap = 64, resort_every = 20;
    bool fp32 = false;  // mixed mode: FP32 particle state, gather, push and march
    std::string err;

    size_t rb() const { return fp32 ? 4 : 8; }

    // mesh (canonical numbering)
    int nn = 0, nt = 0, ne = 0, nf = 0, n_free_e = 0;
    std::vector<int32_t> tet_node, tet_edge, tet_face, tet_nbr, face_edge, edge_lo, edge_hi,
        face_node;
    std::vector<int8_t> tet_esign, tet_fpar, tet_fout, face_esign;
    std::vector<uint8_t> tet_map, edge_free, node_free;
    // device edge numbering: first appearance along the tetrahedron order
    std::vector<int32_t> edev, ecan;  // canonical -> device, device -> canonical
    std::vector<uint32_t> tet_ebase;  // edges first met before tetrahedron t
    std::vector<double> grad, vol;
    Csr meps, mnu, mt;
    double spai_fro = 0;

    // device
    std::vector<void *> allocs;
    int32_t *d_tet_edge = nullptr, *d_fout = nullptr;
    int4 *d_tet_face = nullptr, *d_tet_nbr = nullptr, *d_tet_node = nullptr, *d_face_edge = nullptr;
    uint32_t *d_tet_map = nullptr, *d_tet_ebase = nullptr;
    double *d_grad = nullptr;
    float *d_grad32 = nullptr;
    int2 *d_edge_nodes = nullptr;
    uint8_t *d_edge_free = nullptr;
    int32_t *d_ef_ptr = nullptr, *d_ef_face = nullptr;
    // [*mu^-1] (faces) and M~ (device edge order) in sliced-ELL form
    int32_t *d_nu_sptr = nullptr, *d_nu_sw = nullptr, *d_nu_col = nullptr;
    int32_t *d_mt_sptr = nullptr, *d_mt_sw = nullptr, *d_mt_col = nullptr;
    double *d_nu_val = nullptr, *d_mt_val = nullptr;
    int32_t *d_chunk_sums = nullptr;
    double *d_b = nullptr, *d_bavg = nullptr, *d_h = nullptr, *d_d = nullptr, *d_e = nullptr;
    double *d_cur = nullptr, *d_cur_last = nullptr;
    char *d_rec = nullptr;  // [24 nt] reals of the particle precision
    double *d_b_ext = nullptr, *d_e_ext = nullptr;
    double *d_q = nullptr, *d_divd = nullptr, *d_divb = nullptr;
    unsigned long long *d_counters = nullptr;
    int32_t *d_counts = nullptr, *d_cursor = nullptr;

    // particles (two buffers for the sort; SoA with stride p_cap; reals are
    // double, or float in the mixed mode)
    std::vector<Species3> species;
    int64_t p_cap = 0;
    uint32_t *d_key[2] = {nullptr, nullptr};
    char *d_lam[2] = {nullptr, nullptr}, *d_u[2] = {nullptr, nullptr};  // [3][p_cap] reals
    int32_t *d_pid[2] = {nullptr, nullptr};
    int32_t *d_perm = nullptr;  // [p_cap] sort permutation
    int pbuf = 0;
    // Live count of each species after its last sort, copied by the stream
    // into pinned host memory and applied to Species3::n at the next
    // synchronising call (until then n bounds the live particles from above:
    // the slots past the live ones hold removed keys).
    int32_t *h_alive = nullptr;
    size_t h_alive_cap = 0;
    std::vector<char> alive_pending;

    // state
    int64_t step = 0, steps_since_sort = 0;
    bool have_baseline = false;
    std::vector<double> q0, divd0;

    // stage timing
    uint32_t profile_mask = 0;  // bit k: stage k is timed
    int64_t profile_every = 1;  // on steps that are multiples of this
    std::vector<hipEvent_t> event_pool, all_events;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timed[5];  // recorded, not yet read
    double stage_ms[5] = {0, 0, 0, 0, 0};
    int64_t particle_launches = 0;

    hipEvent_t take_event()
    {
        if (event_pool.empty()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            all_events.push_back(e);
            return e;
        }
        hipEvent_t e = event_pool.back();
        event_pool.pop_back();
        return e;
    }
    // Fold the recorded stage intervals into stage_ms (waits for the last).
    void resolve_timers()
    {
        for (int k = 0; k < 5; ++k) {
            for (auto &ab : timed[k]) {
                float ms = 0;
                if (hipEventSynchronize(ab.second) == hipSuccess &&
                    hipEventElapsedTime(&ms, ab.first, ab.second) == hipSuccess)
                    stage_ms[k] += ms;
                if (k == 1) ++particle_launches;
                event_pool.push_back(ab.first);
                event_pool.push_back(ab.second);
            }
            timed[k].clear();
        }
    }

    fetd_status fail(fetd_status st, const std::string &msg)
    {
        err = msg;
        g_err3 = msg;
        return st;
    }
    fetd_status hip_fail(hipError_t e, const char *where)
    {
        return fail(FETD_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
    }
    template <typename T>
    bool alloc(T **p, size_t count)
    {
        void *q = nullptr;
        if (hipMalloc(&q, std::max<size_t>(1, count) * sizeof(T)) != hipSuccess) return false;
        allocs.push_back(q);
        *p = static_cast<T *>(q);
        return true;
    }
    void release(void *p)
    {
        if (!p) return;
        auto it = std::find(allocs.begin(), allocs.end(), p);
        if (it != allocs.end()) allocs.erase(it);
        (void)hipFree(p);
    }
};

namespace {

template <typename T>
fetd_status upload3(fetd3_sim *s, T **dst, const T *src, size_t count)
{
    if (!*dst && !s->alloc(dst, count)) return s->fail(FETD_E_OOM, "device allocation failed");
    if (count) {
        hipError_t e = hipMemcpyAsync(*dst, src, sizeof(T) * count, hipMemcpyHostToDevice,
                                      s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return s->hip_fail(e, "upload");
    }
    return FETD_OK;
}

template <typename T>
fetd_status zeros3(fetd3_sim *s, T **dst, size_t count)
{
    std::vector<T> z(count, T());
    return upload3(s, dst, z.data(), count);
}

fetd_status download3(fetd3_sim *s, void *dst, const void *src, size_t bytes)
{
    if (!bytes) return FETD_OK;
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "download");
    return FETD_OK;
}

// count reals of the particle precision from the device, as doubles
fetd_status download_reals3(fetd3_sim *s, double *dst, const char *src, int64_t count)
{
    if (!s->fp32) return download3(s, dst, src, 8 * size_t(count));
    std::vector<float> tmp(count);
    fetd_status st = download3(s, tmp.data(), src, 4 * size_t(count));
    if (st) return st;
    for (int64_t i = 0; i < count; ++i) dst[i] = double(tmp[i]);
    return FETD_OK;
}

// Edge arrays cross the boundary in canonical order and live on the device
// in device order.
fetd_status upload_edges3(fetd3_sim *s, double **dst, const double *canon)
{
    std::vector<double> tmp(s->ne);
    for (int r = 0; r < s->ne; ++r) tmp[r] = canon[s->ecan[r]];
    return upload3(s, dst, tmp.data(), tmp.size());
}

fetd_status download_edges3(fetd3_sim *s, double *canon, const double *src)
{
    std::vector<double> tmp(s->ne);
    fetd_status st = download3(s, tmp.data(), src, 8 * tmp.size());
    if (st) return st;
    for (int r = 0; r < s->ne; ++r) canon[s->ecan[r]] = tmp[r];
    return FETD_OK;
}

double det3(const double *a, const double *b, const double *c)
{
    return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
           a[2] * (b[0] * c[1] - b[1] * c[0]);
}

// Topology (edges, faces in lexicographic order of their node ids,
// incidence, neighbours, node maps) and geometry (grad lambda, volumes).
fetd_status build_topology3(fetd3_sim *s, const fetd3_mesh_desc *m)
{
    const int nt = m->n_tets, nn = m->n_nodes;
    s->nt = nt;
    s->nn = nn;
    s->tet_node.assign(m->tet_nodes, m->tet_nodes + 4 * size_t(nt));
    for (int32_t v : s->tet_node)
        if (v < 0 || v >= nn) return s->fail(FETD_E_MESH, "tetrahedron node id out of range");
    // geometry
    s->grad.assign(12 * size_t(nt), 0.0);
    s->vol.assign(nt, 0.0);
    for (int t = 0; t < nt; ++t) {
        double x[4][3];
        for (int k = 0; k < 4; ++k)
            for (int d = 0; d < 3; ++d) {
                x[k][d] = m->node_xyz[3 * size_t(s->tet_node[4 * t + k]) + d];
                if (m->tet_shift && m->period)
                    x[k][d] += double(m->tet_shift[12 * size_t(t) + 3 * k + d]) * m->period[d];
            }
        double J[3][3];  // columns x1-x0, x2-x0, x3-x0
        for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d) J[d][c] = x[c + 1][d] - x[0][d];
        const double c0[3] = {J[0][0], J[1][0], J[2][0]}, c1[3] = {J[0][1], J[1][1], J[2][1]},
                     c2[3] = {J[0][2], J[1][2], J[2][2]};
        const double det = det3(c0, c1, c2);
        if (!(det > 0)) return s->fail(FETD_E_MESH, "tetrahedra must be positively oriented");
        s->vol[t] = det / 6.0;
        // rows of J^-1 = grad lambda_1..3: cofactors / det
        double inv[3][3];
        inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
        inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
        inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
        inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
        double *g = &s->grad[12 * size_t(t)];
        for (int d = 0; d < 3; ++d) {
            g[3 + d] = inv[0][d];
            g[6 + d] = inv[1][d];
            g[9 + d] = inv[2][d];
            g[d] = -(inv[0][d] + inv[1][d] + inv[2][d]);
        }
    }
    // edges
    std::vector<uint64_t> ek(6 * size_t(nt));
    for (int t = 0; t < nt; ++t)
        for (int k = 0; k < 6; ++k) {
            const uint32_t a = s->tet_node[4 * t + LE[k][0]], b = s->tet_node[4 * t + LE[k][1]];
            if (a == b) return s->fail(FETD_E_MESH, "degenerate edge");
            ek[6 * size_t(t) + k] = (uint64_t(std::min(a, b)) << 32) | std::max(a, b);
        }
    std::vector<uint64_t> eu(ek);
    std::sort(eu.begin(), eu.end());
    eu.erase(std::unique(eu.begin(), eu.end()), eu.end());
    s->ne = int(eu.size());
    s->edge_lo.resize(s->ne);
    s->edge_hi.resize(s->ne);
    for (int e = 0; e < s->ne; ++e) {
        s->edge_lo[e] = int32_t(eu[e] >> 32);
        s->edge_hi[e] = int32_t(eu[e] & 0xFFFFFFFFu);
    }
    s->tet_edge.resize(6 * size_t(nt));
    s->tet_esign.resize(6 * size_t(nt));
    for (int t = 0; t < nt; ++t)
        for (int k = 0; k < 6; ++k) {
            const size_t i = 6 * size_t(t) + k;
            s->tet_edge[i] = int32_t(std::lower_bound(eu.begin(), eu.end(), ek[i]) - eu.begin());
            s->tet_esign[i] =
                s->tet_node[4 * t + LE[k][0]] < s->tet_node[4 * t + LE[k][1]] ? 1 : -1;
        }
    // faces: sorted triples
    auto fkey = [](uint32_t a, uint32_t b, uint32_t c) {
        return std::array<uint32_t, 3>{a, b, c};
    };
    std::vector<std::array<uint32_t, 3>> fk(4 * size_t(nt));
    s->tet_fpar.resize(4 * size_t(nt));
    for (int t = 0; t < nt; ++t)
        for (int k = 0; k < 4; ++k) {
            uint32_t v[3] = {uint32_t(s->tet_node[4 * t + LF[k][0]]),
                             uint32_t(s->tet_node[4 * t + LF[k][1]]),
                             uint32_t(s->tet_node[4 * t + LF[k][2]])};
            if (v[0] == v[1] || v[1] == v[2] || v[0] == v[2])
                return s->fail(FETD_E_MESH, "degenerate face");
            // parity of the local order against the sorted order
            int inv = (v[0] > v[1]) + (v[0] > v[2]) + (v[1] > v[2]);
            s->tet_fpar[4 * t + k] = (inv & 1) ? -1 : 1;
            std::sort(v, v + 3);
            fk[4 * size_t(t) + k] = fkey(v[0], v[1], v[2]);
        }
    std::vector<std::array<uint32_t, 3>> fu(fk);
    std::sort(fu.begin(), fu.end());
    fu.erase(std::unique(fu.begin(), fu.end()), fu.end());
    s->nf = int(fu.size());
    s->face_node.resize(3 * size_t(s->nf));
    for (int f = 0; f < s->nf; ++f)
        for (int j = 0; j < 3; ++j) s->face_node[3 * f + j] = int32_t(fu[f][j]);
    s->tet_face.resize(4 * size_t(nt));
    s->tet_fout.resize(4 * size_t(nt));
    std::vector<int32_t> f_t(2 * size_t(s->nf), -1), f_k(2 * size_t(s->nf), -1);
    const int8_t loc_out[4] = {1, -1, 1, -1};
    for (int t = 0; t < nt; ++t)
        for (int k = 0; k < 4; ++k) {
            const size_t i = 4 * size_t(t) + k;
            const int f = int(std::lower_bound(fu.begin(), fu.end(), fk[i]) - fu.begin());
            s->tet_face[i] = f;
            s->tet_fout[i] = int8_t(s->tet_fpar[i] * loc_out[k]);
            if (f_t[2 * f] < 0) {
                f_t[2 * f] = t;
                f_k[2 * f] = k;
            } else if (f_t[2 * f + 1] < 0) {
                f_t[2 * f + 1] = t;
                f_k[2 * f + 1] = k;
            } else {
                return s->fail(FETD_E_MESH, "non-manifold mesh: a face has more than two tetrahedra");
            }
        }
    // neighbours and node maps
    s->tet_nbr.assign(4 * size_t(nt), -1);
    s->tet_map.assign(16 * size_t(nt), 0xFF);
    for (int f = 0; f < s->nf; ++f) {
        if (f_t[2 * f + 1] < 0) continue;
        for (int side = 0; side < 2; ++side) {
            const int t0 = f_t[2 * f + side], k0 = f_k[2 * f + side];
            const int t1 = f_t[2 * f + 1 - side], k1 = f_k[2 * f + 1 - side];
            s->tet_nbr[4 * t0 + k0] = t1;
            for (int j = 0; j < 4; ++j) {
                if (j == k0) continue;
                int hit = -1;
                for (int jj = 0; jj < 4; ++jj)
                    if (s->tet_node[4 * t1 + jj] == s->tet_node[4 * t0 + j]) hit = jj;
                if (hit < 0) return s->fail(FETD_E_MESH, "neighbour node map incomplete");
                s->tet_map[16 * size_t(t0) + 4 * k0 + j] = uint8_t(hit);
            }
            s->tet_map[16 * size_t(t0) + 4 * k0 + k0] = uint8_t(k1);
        }
    }
    // C rows: face (i<j<l) bounds (i,j) +1, (j,l) +1, (i,l) -1
    s->face_edge.resize(3 * size_t(s->nf));
    s->face_esign.resize(3 * size_t(s->nf));
    auto edge_of = [&](uint32_t a, uint32_t b) {
        const uint64_t key = (uint64_t(a) << 32) | b;
        return int32_t(std::lower_bound(eu.begin(), eu.end(), key) - eu.begin());
    };
    for (int f = 0; f < s->nf; ++f) {
        const uint32_t i = fu[f][0], j = fu[f][1], l = fu[f][2];
        s->face_edge[3 * f] = edge_of(i, j);
        s->face_edge[3 * f + 1] = edge_of(j, l);
        s->face_edge[3 * f + 2] = edge_of(i, l);
        s->face_esign[3 * f] = 1;
        s->face_esign[3 * f + 1] = 1;
        s->face_esign[3 * f + 2] = -1;
    }
    // PEC: one-sided faces, their edges and nodes are not free
    s->edge_free.assign(s->ne, 1);
    s->node_free.assign(nn, 1);
    for (int f = 0; f < s->nf; ++f) {
        if (f_t[2 * f + 1] >= 0) continue;
        for (int j = 0; j < 3; ++j) {
            s->edge_free[s->face_edge[3 * f + j]] = 0;
            s->node_free[s->face_node[3 * f + j]] = 0;
        }
    }
    s->n_free_e = 0;
    for (uint8_t v : s->edge_free) s->n_free_e += v;
    return FETD_OK;
}

void csr_from_rows(std::vector<std::vector<std::pair<int, double>>> &rows, Csr &M)
{
    const int n = int(rows.size());
    M.ptr.assign(n + 1, 0);
    M.col.clear();
    M.val.clear();
    for (int r = 0; r < n; ++r) {
        auto &v = rows[r];
        std::stable_sort(v.begin(), v.end(),
                         [](const std::pair<int, double> &a, const std::pair<int, double> &b) {
                             return a.first < b.first;
                         });
        for (size_t i = 0; i < v.size(); ++i) {
            if (M.col.size() > size_t(M.ptr[r]) && M.col.back() == v[i].first)
                M.val.back() += v[i].second;
            else {
                M.col.push_back(v[i].first);
                M.val.push_back(v[i].second);
            }
        }
        M.ptr[r + 1] = int32_t(M.col.size());
    }
}

inline double lmass(double V, int p, int q) { return V * (p == q ? 2.0 : 1.0) / 20.0; }

// [*eps]_ij = eps0 int W1_i . W1_j (free edges; wall rows are the identity)
// and [*mu^-1]_fg = (1/mu0) int W2_f . W2_g, from int l_p l_q = V(1+d_pq)/20.
void assemble_hodges3(fetd3_sim *s)
{
    std::vector<std::vector<std::pair<int, double>>> re(s->ne), rf(s->nf);
    for (int t = 0; t < s->nt; ++t) {
        const double *g = &s->grad[12 * size_t(t)];
        const double V = s->vol[t];
        auto gd = [&](int p, int q) {
            return g[3 * p] * g[3 * q] + g[3 * p + 1] * g[3 * q + 1] + g[3 * p + 2] * g[3 * q + 2];
        };
        for (int k = 0; k < 6; ++k) {
            const int ek = s->tet_edge[6 * t + k];
            if (!s->edge_free[ek]) continue;
            const int a = LE[k][0], b = LE[k][1];
            for (int l = 0; l < 6; ++l) {
                const int el = s->tet_edge[6 * t + l];
                if (!s->edge_free[el]) continue;
                const int c = LE[l][0], d = LE[l][1];
                const double v = gd(b, d) * lmass(V, a, c) - gd(b, c) * lmass(V, a, d) -
                                 gd(a, d) * lmass(V, b, c) + gd(a, c) * lmass(V, b, d);
                re[ek].push_back({el, s->eps0 * double(s->tet_esign[6 * t + k]) *
                                          double(s->tet_esign[6 * t + l]) * v});
            }
        }
        // W2 of local face k = 2 sum_n l_n Y[k][n]
        double Y[4][4][3] = {};
        for (int k = 0; k < 4; ++k) {
            const int p = LF[k][0], q = LF[k][1], r = LF[k][2];
            auto cr = [&](int a, int b, double *o) {
                o[0] = g[3 * a + 1] * g[3 * b + 2] - g[3 * a + 2] * g[3 * b + 1];
                o[1] = g[3 * a + 2] * g[3 * b] - g[3 * a] * g[3 * b + 2];
                o[2] = g[3 * a] * g[3 * b + 1] - g[3 * a + 1] * g[3 * b];
            };
            cr(q, r, Y[k][p]);
            cr(r, p, Y[k][q]);
            cr(p, q, Y[k][r]);
        }
        for (int k = 0; k < 4; ++k)
            for (int l = 0; l < 4; ++l) {
                double acc = 0.0;
                for (int p = 0; p < 4; ++p)
                    for (int q = 0; q < 4; ++q)
                        acc += lmass(V, p, q) * (Y[k][p][0] * Y[l][q][0] + Y[k][p][1] * Y[l][q][1] +
                                                 Y[k][p][2] * Y[l][q][2]);
                rf[s->tet_face[4 * t + k]].push_back(
                    {s->tet_face[4 * t + l], 4.0 * double(s->tet_fpar[4 * t + k]) *
                                                 double(s->tet_fpar[4 * t + l]) * acc / s->mu0});
            }
    }
    for (int e = 0; e < s->ne; ++e)
        if (!s->edge_free[e]) re[e].push_back({e, 1.0});
    csr_from_rows(re, s->meps);
    csr_from_rows(rf, s->mnu);
}

// Sliced-ELL copy of a CSR matrix (rows in the given order, entries in
// their stored order; padding value 0 with the row itself as column).
struct SellHost {
    std::vector<int32_t> sptr, sw, col;
    std::vector<double> val;
};

SellHost to_sell(const std::vector<int32_t> &ptr, const std::vector<int32_t> &col,
                 const std::vector<double> &val)
{
    SellHost h;
    const int n = int(ptr.size()) - 1;
    const int ns = (n + 63) / 64;
    h.sptr.resize(ns);
    h.sw.resize(ns);
    int64_t off = 0;
    for (int sl = 0; sl < ns; ++sl) {
        int w = 0;
        for (int r = 64 * sl; r < std::min(n, 64 * sl + 64); ++r) w = std::max(w, ptr[r + 1] - ptr[r]);
        h.sptr[sl] = int32_t(off);
        h.sw[sl] = w;
        off += int64_t(w) * 64;
    }
    h.col.assign(off, 0);
    h.val.assign(off, 0.0);
    for (int sl = 0; sl < ns; ++sl)
        for (int lane = 0; lane < 64; ++lane) {
            const int r = 64 * sl + lane;
            for (int j = 0; j < h.sw[sl]; ++j) {
                const int64_t q = h.sptr[sl] + 64 * j + lane;
                if (r < n && j < ptr[r + 1] - ptr[r]) {
                    h.col[q] = col[ptr[r] + j];
                    h.val[q] = val[ptr[r] + j];
                } else {
                    h.col[q] = r < n ? r : 0;
                }
            }
        }
    return h;
}

// Device edge numbering by first appearance along the tetrahedron order:
// the edges of a run of consecutive tetrahedra get nearby ids, so one
// particle block's currents fall into a short window of ids.
void number_edges3(fetd3_sim *s)
{
    s->edev.assign(s->ne, -1);
    s->ecan.assign(s->ne, -1);
    s->tet_ebase.assign(s->nt, 0);
    int32_t next = 0;
    for (int t = 0; t < s->nt; ++t) {
        s->tet_ebase[t] = uint32_t(next);
        for (int k = 0; k < 6; ++k) {
            const int e = s->tet_edge[6 * t + k];
            if (s->edev[e] < 0) {
                s->edev[e] = next;
                s->ecan[next] = e;
                ++next;
            }
        }
    }
}

fetd_status upload_mesh3(fetd3_sim *s)
{
    fetd_status st;
    const int nt = s->nt, nf = s->nf, ne = s->ne;
    number_edges3(s);
    const std::vector<int32_t> &edev = s->edev, &ecan = s->ecan;
    std::vector<int32_t> te(8 * size_t(nt), 0), fout(nt, 0);
    std::vector<int4> tf(nt), tn(nt), tnode(nt), fe(nf);
    std::vector<uint32_t> tm(nt, 0);
    for (int t = 0; t < nt; ++t) {
        int bits = 0;
        for (int k = 0; k < 6; ++k) {
            te[8 * size_t(t) + k] = edev[s->tet_edge[6 * t + k]];
            if (s->tet_esign[6 * t + k] < 0) bits |= 1 << k;
        }
        for (int k = 0; k < 4; ++k) {
            if (s->tet_fpar[4 * t + k] < 0) bits |= 1 << (8 + k);
            if (s->tet_fout[4 * t + k] < 0) fout[t] |= 1 << k;
        }
        te[8 * size_t(t) + 6] = bits;
        tf[t] = make_int4(s->tet_face[4 * t], s->tet_face[4 * t + 1], s->tet_face[4 * t + 2],
                          s->tet_face[4 * t + 3]);
        tn[t] = make_int4(s->tet_nbr[4 * t], s->tet_nbr[4 * t + 1], s->tet_nbr[4 * t + 2],
                          s->tet_nbr[4 * t + 3]);
        tnode[t] = make_int4(s->tet_node[4 * t], s->tet_node[4 * t + 1], s->tet_node[4 * t + 2],
                             s->tet_node[4 * t + 3]);
        uint32_t m = 0;
        for (int k = 0; k < 4; ++k) {
            if (s->tet_nbr[4 * t + k] < 0) continue;
            const uint8_t *mp = &s->tet_map[16 * size_t(t) + 4 * k];
            const uint32_t byte = uint32_t(mp[(k + 1) & 3]) | (uint32_t(mp[(k + 2) & 3]) << 2) |
                                  (uint32_t(mp[(k + 3) & 3]) << 4) | (uint32_t(mp[k]) << 6);
            m |= byte << (8 * k);
        }
        tm[t] = m;
    }
    for (int f = 0; f < nf; ++f) {
        int bits = 0;
        for (int j = 0; j < 3; ++j)
            if (s->face_esign[3 * f + j] < 0) bits |= 1 << j;
        fe[f] = make_int4(edev[s->face_edge[3 * f]], edev[s->face_edge[3 * f + 1]],
                          edev[s->face_edge[3 * f + 2]], bits);
    }
    // edge -> faces (C^T) in device edge order, faces in increasing order,
    // sign in bit 31
    std::vector<int32_t> efp(ne + 1, 0), eff;
    for (int f = 0; f < nf; ++f)
        for (int j = 0; j < 3; ++j) ++efp[edev[s->face_edge[3 * f + j]] + 1];
    for (int e = 0; e < ne; ++e) efp[e + 1] += efp[e];
    eff.resize(efp[ne]);
    {
        std::vector<int32_t> pos(efp.begin(), efp.end() - 1);
        for (int f = 0; f < nf; ++f)
            for (int j = 0; j < 3; ++j) {
                const int r = edev[s->face_edge[3 * f + j]];
                eff[pos[r]++] = s->face_esign[3 * f + j] < 0 ? int32_t(uint32_t(f) | 0x80000000u) : f;
            }
    }
    std::vector<int2> en(ne);
    std::vector<uint8_t> efree(ne);
    for (int r = 0; r < ne; ++r) {
        en[r] = make_int2(s->edge_lo[ecan[r]], s->edge_hi[ecan[r]]);
        efree[r] = s->edge_free[ecan[r]];
    }
    // M~ in device order; each row keeps the canonical order of its entries
    std::vector<int32_t> mtp(ne + 1, 0), mtc;
    std::vector<double> mtv;
    mtc.reserve(s->mt.col.size());
    mtv.reserve(s->mt.val.size());
    for (int r = 0; r < ne; ++r) {
        const int e = ecan[r];
        for (int q = s->mt.ptr[e]; q < s->mt.ptr[e + 1]; ++q) {
            mtc.push_back(edev[s->mt.col[q]]);
            mtv.push_back(s->mt.val[q]);
        }
        mtp[r + 1] = int32_t(mtc.size());
    }
    if ((st = upload3(s, &s->d_tet_edge, te.data(), te.size()))) return st;
    if ((st = upload3(s, &s->d_fout, fout.data(), fout.size()))) return st;
    if ((st = upload3(s, &s->d_tet_face, tf.data(), tf.size()))) return st;
    if ((st = upload3(s, &s->d_tet_nbr, tn.data(), tn.size()))) return st;
    if ((st = upload3(s, &s->d_tet_node, tnode.data(), tnode.size()))) return st;
    if ((st = upload3(s, &s->d_tet_map, tm.data(), tm.size()))) return st;
    if ((st = upload3(s, &s->d_grad, s->grad.data(), s->grad.size()))) return st;
    {
        std::vector<float> g32(s->grad.begin(), s->grad.end());
        if ((st = upload3(s, &s->d_grad32, g32.data(), g32.size()))) return st;
    }
    if ((st = upload3(s, &s->d_face_edge, fe.data(), fe.size()))) return st;
    if ((st = upload3(s, &s->d_ef_ptr, efp.data(), efp.size()))) return st;
    if ((st = upload3(s, &s->d_ef_face, eff.data(), eff.size()))) return st;
    if ((st = upload3(s, &s->d_edge_nodes, en.data(), en.size()))) return st;
    if ((st = upload3(s, &s->d_edge_free, efree.data(), efree.size()))) return st;
    if ((st = upload3(s, &s->d_tet_ebase, s->tet_ebase.data(), s->tet_ebase.size()))) return st;
    {
        const SellHost nu = to_sell(s->mnu.ptr, s->mnu.col, s->mnu.val);
        const SellHost mt = to_sell(mtp, mtc, mtv);
        if ((st = upload3(s, &s->d_nu_sptr, nu.sptr.data(), nu.sptr.size()))) return st;
        if ((st = upload3(s, &s->d_nu_sw, nu.sw.data(), nu.sw.size()))) return st;
        if ((st = upload3(s, &s->d_nu_col, nu.col.data(), nu.col.size()))) return st;
        if ((st = upload3(s, &s->d_nu_val, nu.val.data(), nu.val.size()))) return st;
        if ((st = upload3(s, &s->d_mt_sptr, mt.sptr.data(), mt.sptr.size()))) return st;
        if ((st = upload3(s, &s->d_mt_sw, mt.sw.data(), mt.sw.size()))) return st;
        if ((st = upload3(s, &s->d_mt_col, mt.col.data(), mt.col.size()))) return st;
        if ((st = upload3(s, &s->d_mt_val, mt.val.data(), mt.val.size()))) return st;
    }
    if ((st = zeros3(s, &s->d_chunk_sums, size_t(nt + 1 + 1023) / 1024 + 1))) return st;
    if ((st = zeros3(s, &s->d_b, nf)) || (st = zeros3(s, &s->d_bavg, nf)) ||
        (st = zeros3(s, &s->d_h, nf)) || (st = zeros3(s, &s->d_d, ne)) ||
        (st = zeros3(s, &s->d_e, ne)) || (st = zeros3(s, &s->d_cur, ne)) ||
        (st = zeros3(s, &s->d_cur_last, ne)) || (st = zeros3(s, &s->d_rec, size_t(kRec) * nt * s->rb())) ||
        (st = zeros3(s, &s->d_q, s->nn)) || (st = zeros3(s, &s->d_divd, s->nn)) ||
        (st = zeros3(s, &s->d_divb, nt)) || (st = zeros3(s, &s->d_counters, 4)) ||
        (st = zeros3(s, &s->d_counts, size_t(nt) + 1)) ||
        (st = zeros3(s, &s->d_cursor, size_t(nt) + 1)))
        return st;
    unsigned long long init[4] = {0, 0, 0, ~0ull};
    return upload3(s, &s->d_counters, init, 4);
}

Sell mt_sell(const fetd3_sim *s) { return Sell{s->d_mt_sptr, s->d_mt_sw, s->d_mt_col, s->d_mt_val}; }
Sell nu_sell(const fetd3_sim *s) { return Sell{s->d_nu_sptr, s->d_nu_sw, s->d_nu_col, s->d_nu_val}; }

Mesh3 mesh_view(const fetd3_sim *s)
{
    Mesh3 m;
    m.tet_edge = s->d_tet_edge;
    m.tet_face = s->d_tet_face;
    m.tet_nbr = s->d_tet_nbr;
    m.tet_map = s->d_tet_map;
    m.grad = s->d_grad;
    m.grad32 = s->d_grad32;
    m.tet_ebase = s->d_tet_ebase;
    return m;
}

fetd_status check_errors3(fetd3_sim *s)
{
    unsigned long long c[4];
    fetd_status st = download3(s, c, s->d_counters, sizeof c);  // synchronises
    if (st) return st;
    for (size_t i = 0; i < s->alive_pending.size() && i < s->species.size(); ++i)
        if (s->alive_pending[i]) {
            s->species[i].n = s->h_alive[i];
            s->alive_pending[i] = 0;
        }
    if (c[2]) {
        return s->fail(FETD_E_TRACK, std::string(c[2] & 1 ? "crossing cap exceeded" :
                                                              "non-finite momentum") +
                                         " (particle slot " + std::to_string(c[3]) + ")");
    }
    return FETD_OK;
}

fetd_status compute_charge3(fetd3_sim *s)
{
    hipError_t e = hipMemsetAsync(s->d_q, 0, sizeof(double) * s->nn, s->stream);
    for (const Species3 &sp : s->species) {
        if (e != hipSuccess) break;
        e = launch3_charge(s->stream, sp.n, s->d_key[s->pbuf] + sp.offset,
                           s->d_lam[s->pbuf] + sp.offset * s->rb(), s->fp32, s->p_cap,
                           s->d_tet_node, sp.q * sp.w, s->d_q);
    }
    if (e != hipSuccess) return s->hip_fail(e, "charge");
    return FETD_OK;
}

fetd_status compute_divd3(fetd3_sim *s)
{
    hipError_t e = hipMemsetAsync(s->d_divd, 0, sizeof(double) * s->nn, s->stream);
    if (e == hipSuccess) e = launch3_divd(s->stream, s->ne, s->d_edge_nodes, s->d_d, s->d_divd);
    if (e != hipSuccess) return s->hip_fail(e, "divd");
    return FETD_OK;
}

fetd_status take_baseline3(fetd3_sim *s)
{
    fetd_status st;
    if ((st = compute_charge3(s)) || (st = compute_divd3(s))) return st;
    s->q0.resize(s->nn);
    s->divd0.resize(s->nn);
    if ((st = download3(s, s->q0.data(), s->d_q, 8 * size_t(s->nn)))) return st;
    if ((st = download3(s, s->divd0.data(), s->d_divd, 8 * size_t(s->nn)))) return st;
    s->have_baseline = true;
    return FETD_OK;
}

// Grow both particle buffers to hold `extra` more particles.
fetd_status grow_particles3(fetd3_sim *s, int64_t extra)
{
    int64_t used = 0;
    for (const Species3 &sp : s->species) used = std::max(used, sp.offset + sp.n);
    const int64_t need = used + extra;
    if (need <= s->p_cap) return FETD_OK;
    const int64_t cap = std::max<int64_t>(need, s->p_cap + s->p_cap / 2);
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "grow");
    for (int b = 0; b < 2; ++b) {
        const size_t rb = s->rb();
        uint32_t *key = nullptr;
        char *lam = nullptr, *u = nullptr;
        int32_t *pid = nullptr;
        if (!s->alloc(&key, cap) || !s->alloc(&lam, 3 * cap * rb) || !s->alloc(&u, 3 * cap * rb) ||
            !s->alloc(&pid, cap))
            return s->fail(FETD_E_OOM, "particle allocation failed");
        e = hipMemsetAsync(key, 0xFF, sizeof(uint32_t) * cap, s->stream);
        if (used > 0 && e == hipSuccess) {
            e = hipMemcpyAsync(key, s->d_key[b], 4 * used, hipMemcpyDeviceToDevice, s->stream);
            for (int c = 0; c < 3 && e == hipSuccess; ++c) {
                e = hipMemcpyAsync(lam + c * cap * rb, s->d_lam[b] + c * s->p_cap * rb, rb * used,
                                   hipMemcpyDeviceToDevice, s->stream);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(u + c * cap * rb, s->d_u[b] + c * s->p_cap * rb, rb * used,
                                       hipMemcpyDeviceToDevice, s->stream);
            }
            if (e == hipSuccess)
                e = hipMemcpyAsync(pid, s->d_pid[b], 4 * used, hipMemcpyDeviceToDevice, s->stream);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return s->hip_fail(e, "grow copy");
        s->release(s->d_key[b]);
        s->release(s->d_lam[b]);
        s->release(s->d_u[b]);
        s->release(s->d_pid[b]);
        s->d_key[b] = key;
        s->d_lam[b] = lam;
        s->d_u[b] = u;
        s->d_pid[b] = pid;
    }
    s->release(s->d_perm);
    s->d_perm = nullptr;
    if (!s->alloc(&s->d_perm, cap)) return s->fail(FETD_E_OOM, "particle allocation failed");
    s->p_cap = cap;
    return FETD_OK;
}

fetd_status sort_all3(fetd3_sim *s)
{
    const int cb = s->pbuf, ob = 1 - s->pbuf;
    if (s->h_alive_cap < s->species.size()) {
        // a copy into the old buffer may be in flight
        hipError_t e = hipStreamSynchronize(s->stream);
        if (e == hipSuccess && s->h_alive) e = hipHostFree(s->h_alive);
        s->h_alive = nullptr;
        s->h_alive_cap = 0;
        s->alive_pending.clear();
        const size_t cap = std::max<size_t>(16, 2 * s->species.size());
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void **>(&s->h_alive), sizeof(int32_t) * cap,
                              hipHostMallocDefault);
        if (e != hipSuccess) return s->hip_fail(e, "sort");
        s->h_alive_cap = cap;
        s->alive_pending.assign(cap, 0);
    }
    for (size_t si = 0; si < s->species.size(); ++si) {
        Species3 &sp = s->species[si];
        if (sp.n == 0) continue;
        Sort3 a;
        a.n = sp.n;
        a.nt = s->nt;
        a.key_in = s->d_key[cb] + sp.offset;
        a.lam_in = s->d_lam[cb] + sp.offset * s->rb();
        a.u_in = s->d_u[cb] + sp.offset * s->rb();
        a.pid_in = s->d_pid[cb] + sp.offset;
        a.key_out = s->d_key[ob] + sp.offset;
        a.lam_out = s->d_lam[ob] + sp.offset * s->rb();
        a.u_out = s->d_u[ob] + sp.offset * s->rb();
        a.elem_bytes = int(s->rb());
        a.pid_out = s->d_pid[ob] + sp.offset;
        a.stride_in = a.stride_out = s->p_cap;
        a.counts = s->d_counts;
        a.cursor = s->d_cursor;
        a.chunk_sums = s->d_chunk_sums;
        a.perm = s->d_perm + sp.offset;
        // the tail beyond the live particles keeps lost keys
        hipError_t e = hipMemsetAsync(a.key_out, 0xFF, 4 * size_t(sp.n), s->stream);
        if (e == hipSuccess) e = launch3_sort(s->stream, a);
        // cursor[nt] ends at the total of live particles
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->h_alive + si, s->d_cursor + s->nt, 4, hipMemcpyDeviceToHost,
                               s->stream);
        if (e != hipSuccess) return s->hip_fail(e, "sort");
        s->alive_pending[si] = 1;
    }
    s->pbuf = ob;
    s->steps_since_sort = 0;
    return FETD_OK;
}

// Stage interval of the profiled stream, read later (no wait inside the
// step loop).  The step stages (0-3) hand their two events to the stage's
// kernel launches, which carry them in their own dispatches; the sort (4)
// records them around its launches.
struct StageTimer3 {
    fetd3_sim *s;
    int k;
    hipEvent_t a = nullptr, b = nullptr;
    StageTimer3(fetd3_sim *sim, int stage) : s(sim), k(stage)
    {
        if (!(s->profile_mask >> k & 1u) || s->step % s->profile_every != 0) return;
        a = s->take_event();
        b = a ? s->take_event() : nullptr;
        if (!b) {
            release();
            return;
        }
        if (k == 4) {
            if (hipEventRecord(a, s->stream) != hipSuccess) release();
        } else {
            fetd_timing::pending() = {a, b};
        }
    }
    void release()
    {
        if (a) s->event_pool.push_back(a);
        if (b) s->event_pool.push_back(b);
        a = b = nullptr;
    }
    ~StageTimer3()
    {
        if (!a) return;
        bool ok;
        if (k == 4) {
            ok = hipEventRecord(b, s->stream) == hipSuccess;
        } else {
            ok = fetd_timing::pending().start == nullptr;  // a kernel took the events
            fetd_timing::pending() = {};
        }
        if (ok)
            s->timed[k].push_back({a, b});
        else
            release();
    }
};

}  // namespace

extern "C" {

fetd_status fetd3_mesh_create(const fetd3_mesh_desc *mesh, const fetd3_opts *opts,
                              fetd3_sim **out)
{
    if (!out) {
        g_err3 = "out is NULL";
        return FETD_E_ARG;
    }
    *out = nullptr;
    if (!mesh || !opts || !mesh->node_xyz || !mesh->tet_nodes || mesh->n_nodes <= 0 ||
        mesh->n_tets <= 0 || mesh->n_tets > int32_t(kTetMask) || !(opts->dt > 0) ||
        !(opts->eps0 > 0) || !(opts->mu0 > 0) || !(opts->c > 0) || opts->spai_level < 0 ||
        opts->spai_level > 2 || (mesh->tet_shift && !mesh->period) ||
        (opts->precision != FETD_FP64 && opts->precision != FETD_MIXED)) {
        g_err3 = "invalid mesh description or options";
        return FETD_E_ARG;
    }
    fetd3_sim *s = new (std::nothrow) fetd3_sim();
    if (!s) return FETD_E_OOM;
    s->device = opts->device;
    s->dt = opts->dt;
    s->eps0 = opts->eps0;
    s->mu0 = opts->mu0;
    s->c = opts->c;
    s->spai_level = opts->spai_level;
    s->cap = opts->crossing_cap > 0 ? opts->crossing_cap : 64;
    s->resort_every = opts->resort_every > 0 ? opts->resort_every : 20;
    s->fp32 = opts->precision == FETD_MIXED;
    DeviceGuard3 g(s->device);
    fetd_status st = build_topology3(s, mesh);
    if (!st) {
        assemble_hodges3(s);
        if (!fetd::spai_build(s->meps, s->edge_free.data(), s->spai_level, s->mt))
            st = s->fail(FETD_E_MESH, "SPAI normal equations not positive definite");
        else
            s->spai_fro = fetd::spai_frobenius(s->meps, s->mt, s->edge_free.data(), s->n_free_e);
    }
    if (!st) {
        if (opts->hip_stream) {
            s->stream = static_cast<hipStream_t>(opts->hip_stream);
        } else {
            hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
            if (e != hipSuccess) st = s->hip_fail(e, "stream");
            s->own_stream = true;
        }
    }
    if (!st) st = upload_mesh3(s);
    if (st) {
        g_err3 = s->err;
        fetd3_destroy(s);
        return st;
    }
    *out = s;
    return FETD_OK;
}

fetd_status fetd3_fields_set(fetd3_sim *s, const double *b_ext, const double *e_ext)
{
    if (!s) return FETD_E_ARG;
    DeviceGuard3 g(s->device);
    if (hipError_t e = hipStreamSynchronize(s->stream)) return s->hip_fail(e, "fields_set");
    fetd_status st;
    if (b_ext) {
        if ((st = upload3(s, &s->d_b_ext, b_ext, 3 * size_t(s->nt)))) return st;
    } else {
        s->release(s->d_b_ext);
        s->d_b_ext = nullptr;
    }
    if (e_ext) {
        if ((st = upload_edges3(s, &s->d_e_ext, e_ext))) return st;
    } else {
        s->release(s->d_e_ext);
        s->d_e_ext = nullptr;
    }
    return FETD_OK;
}

fetd_status fetd3_fields_load(fetd3_sim *s, const double *b, const double *d)
{
    if (!s) return FETD_E_ARG;
    DeviceGuard3 g(s->device);
    if (b)
        for (int f = 0; f < s->nf; ++f)
            if (!std::isfinite(b[f])) return s->fail(FETD_E_ARG, "b must be finite");
    if (d)
        for (int e = 0; e < s->ne; ++e)
            if (!std::isfinite(d[e])) return s->fail(FETD_E_ARG, "d must be finite");
    if (hipError_t e = hipStreamSynchronize(s->stream)) return s->hip_fail(e, "fields_load");
    fetd_status st;
    if (b && (st = upload3(s, &s->d_b, b, size_t(s->nf)))) return st;
    if (d) {
        std::vector<double> df(d, d + s->ne);
        for (int e = 0; e < s->ne; ++e)
            if (!s->edge_free[e]) df[e] = 0.0;
        if ((st = upload_edges3(s, &s->d_d, df.data()))) return st;
        hipError_t e = launch3_spmv(s->stream, s->ne, mt_sell(s), s->d_edge_free, s->d_d, s->d_e);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return s->hip_fail(e, "fields_load spmv");
    }
    s->have_baseline = false;
    return FETD_OK;
}

fetd_status fetd3_particles_load_bary(fetd3_sim *s, double q, double m, double w, int64_t n,
                                      const int32_t *tet, const int8_t *slot, const double *lam,
                                      const double *u, int32_t *species_out)
{
    if (!s) return FETD_E_ARG;
    if (n < 0 || (n > 0 && (!tet || !lam || !u)) || !(m > 0) || n > (int64_t(1) << 31) - 1)
        return s->fail(FETD_E_ARG, "invalid particle arguments");
    for (int64_t i = 0; i < n; ++i) {
        if (tet[i] < 0 || tet[i] >= s->nt) return s->fail(FETD_E_ARG, "tetrahedron id out of range");
        if (slot && (slot[i] < 0 || slot[i] > 3)) return s->fail(FETD_E_ARG, "slot out of range");
    }
    DeviceGuard3 g(s->device);
    fetd_status st = grow_particles3(s, n);
    if (st) return st;
    int64_t used = 0;
    for (const Species3 &sp : s->species) used = std::max(used, sp.offset + sp.n);
    Species3 sp;
    sp.q = q;
    sp.m = m;
    sp.w = w;
    sp.n = sp.n_loaded = n;
    sp.offset = used;
    if (n > 0) {
        std::vector<uint32_t> key(n);
        std::vector<int32_t> pid(n);
        const size_t rb = s->rb();
        std::vector<char> L(3 * n * rb), U(3 * n * rb);
        for (int64_t i = 0; i < n; ++i) {
            key[i] = uint32_t(tet[i]) | (uint32_t(slot ? slot[i] : 0) << 30);
            pid[i] = int32_t(i);
            for (int c = 0; c < 3; ++c) {
                if (s->fp32) {
                    reinterpret_cast<float *>(L.data())[c * n + i] = float(lam[3 * i + c]);
                    reinterpret_cast<float *>(U.data())[c * n + i] = float(u[3 * i + c]);
                } else {
                    reinterpret_cast<double *>(L.data())[c * n + i] = lam[3 * i + c];
                    reinterpret_cast<double *>(U.data())[c * n + i] = u[3 * i + c];
                }
            }
        }
        const int b = s->pbuf;
        hipError_t e = hipMemcpyAsync(s->d_key[b] + used, key.data(), 4 * n,
                                      hipMemcpyHostToDevice, s->stream);
        for (int c = 0; c < 3 && e == hipSuccess; ++c) {
            e = hipMemcpyAsync(s->d_lam[b] + (c * s->p_cap + used) * rb, &L[c * n * rb], rb * n,
                               hipMemcpyHostToDevice, s->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(s->d_u[b] + (c * s->p_cap + used) * rb, &U[c * n * rb], rb * n,
                                   hipMemcpyHostToDevice, s->stream);
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->d_pid[b] + used, pid.data(), 4 * n, hipMemcpyHostToDevice,
                               s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return s->hip_fail(e, "particle upload");
    }
    s->species.push_back(sp);
    if (species_out) *species_out = int32_t(s->species.size() - 1);
    s->have_baseline = false;
    // start sorted by tetrahedron (the particle kernel's locality relies on it)
    if (n > 0) return sort_all3(s);
    return FETD_OK;
}

fetd_status fetd3_pic_step(fetd3_sim *s, int32_t n_steps, int32_t pusher)
{
    if (!s || n_steps < 0 || pusher < 0 || pusher > 3) return FETD_E_ARG;
    DeviceGuard3 g(s->device);
    fetd_status st;
    if (!s->have_baseline && (st = take_baseline3(s))) return st;
    const Mesh3 mv = mesh_view(s);
    for (int it = 0; it < n_steps; ++it) {
        if (s->steps_since_sort >= s->resort_every) {
            StageTimer3 tm(s, 4);
            if ((st = sort_all3(s))) return st;
        }
        hipError_t e;
        {
            StageTimer3 tm(s, 0);
            e = launch3_faraday(s->stream, s->nf, s->d_face_edge, s->d_e, s->d_b, s->d_bavg, s->dt);
            if (e == hipSuccess)
                e = launch3_record(s->stream, s->nt, mv, s->d_e, s->d_e_ext, s->d_bavg, s->d_rec,
                                   s->fp32);
        }
        if (e != hipSuccess) return s->hip_fail(e, "faraday");
        for (const Species3 &sp : s->species) {
            Step3 a;
            a.n = sp.n;
            a.key = s->d_key[s->pbuf] + sp.offset;
            a.lam = s->d_lam[s->pbuf] + sp.offset * s->rb();
            a.u = s->d_u[s->pbuf] + sp.offset * s->rb();
            a.rec = s->d_rec;
            a.b_ext = s->d_b_ext;
            a.cur = s->d_cur;
            a.qdt = sp.q * sp.w / s->dt;
            a.alpha = sp.q * s->dt / (2.0 * sp.m);
            a.dt = s->dt;
            a.c = s->c;
            a.inv_c2 = 1.0 / (s->c * s->c);
            a.cap = s->cap;
            a.counters = s->d_counters;
            a.stride = s->p_cap;
            StageTimer3 tm(s, 1);
            e = launch3_particles(s->stream, mv, a, pusher, s->fp32);
            if (e != hipSuccess) return s->hip_fail(e, "particles");
        }
        {
            StageTimer3 tm(s, 2);
            e = launch3_hnu(s->stream, s->nf, nu_sell(s), s->d_b, s->d_h);
            if (e == hipSuccess)
                e = launch3_ampere(s->stream, s->ne, s->d_ef_ptr, s->d_ef_face, s->d_edge_free,
                                   s->d_h, s->d_cur, s->d_cur_last, s->d_d, s->dt);
        }
        if (e != hipSuccess) return s->hip_fail(e, "ampere");
        {
            StageTimer3 tm(s, 3);
            e = launch3_spmv(s->stream, s->ne, mt_sell(s), s->d_edge_free, s->d_d, s->d_e);
        }
        if (e != hipSuccess) return s->hip_fail(e, "spmv");
        ++s->step;
        ++s->steps_since_sort;
    }
    return FETD_OK;
}

fetd_status fetd3_sort(fetd3_sim *s)
{
    if (!s) return FETD_E_ARG;
    DeviceGuard3 g(s->device);
    return sort_all3(s);
}

fetd_status fetd3_sync(fetd3_sim *s)
{
    if (!s) return FETD_E_ARG;
    DeviceGuard3 g(s->device);
    return check_errors3(s);
}

fetd_status fetd3_fields_get(fetd3_sim *s, int32_t which, void *dst, int64_t capacity,
                             int64_t *written)
{
    if (!s) return FETD_E_ARG;
    DeviceGuard3 g(s->device);
    fetd_status st = check_errors3(s);
    if (st) return st;
    const void *src = nullptr;
    size_t bytes = 0;
    bool host = false, edge = false;
    std::vector<int32_t> tmp;
    hipError_t e = hipSuccess;
    switch (which) {
    case FETD3_FIELD_E: src = s->d_e; bytes = 8 * size_t(s->ne); edge = true; break;
    case FETD3_FIELD_D: src = s->d_d; bytes = 8 * size_t(s->ne); edge = true; break;
    case FETD3_FIELD_B: src = s->d_b; bytes = 8 * size_t(s->nf); break;
    case FETD3_FIELD_J: src = s->d_cur_last; bytes = 8 * size_t(s->ne); edge = true; break;
    case FETD3_FIELD_Q:
        if ((st = compute_charge3(s))) return st;
        src = s->d_q;
        bytes = 8 * size_t(s->nn);
        break;
    case FETD3_FIELD_DIVD:
        if ((st = compute_divd3(s))) return st;
        src = s->d_divd;
        bytes = 8 * size_t(s->nn);
        break;
    case FETD3_FIELD_DIVB:
        e = launch3_divb(s->stream, s->nt, s->d_tet_face, s->d_fout, s->d_b, s->d_divb);
        if (e != hipSuccess) return s->hip_fail(e, "divb");
        src = s->d_divb;
        bytes = 8 * size_t(s->nt);
        break;
    case FETD3_FIELD_EDGES:
        tmp.resize(2 * size_t(s->ne));
        for (int i = 0; i < s->ne; ++i) {
            tmp[2 * i] = s->edge_lo[i];
            tmp[2 * i + 1] = s->edge_hi[i];
        }
        src = tmp.data();
        bytes = 4 * tmp.size();
        host = true;
        break;
    case FETD3_FIELD_FACES: src = s->face_node.data(); bytes = 4 * s->face_node.size(); host = true; break;
    case FETD3_FIELD_SPAI_PTR: src = s->mt.ptr.data(); bytes = 4 * s->mt.ptr.size(); host = true; break;
    case FETD3_FIELD_SPAI_COL: src = s->mt.col.data(); bytes = 4 * s->mt.col.size(); host = true; break;
    case FETD3_FIELD_SPAI_VAL: src = s->mt.val.data(); bytes = 8 * s->mt.val.size(); host = true; break;
    default: return s->fail(FETD_E_ARG, "unknown field selector");
    }
    if (written) *written = int64_t(bytes);
    if (!dst) return FETD_OK;
    if (capacity < int64_t(bytes)) return s->fail(FETD_E_ARG, "capacity too small");
    if (host) {
        std::memcpy(dst, src, bytes);
        return FETD_OK;
    }
    if (edge) return download_edges3(s, static_cast<double *>(dst), static_cast<const double *>(src));
    return download3(s, dst, src, bytes);
}

fetd_status fetd3_particles_get(fetd3_sim *s, int32_t species, int64_t capacity, int32_t *tet,
                                int8_t *slot, double *lam, double *u, int32_t *id,
                                int64_t *n_out)
{
    if (!s || species < 0 || species >= int32_t(s->species.size())) return FETD_E_ARG;
    DeviceGuard3 g(s->device);
    fetd_status st = check_errors3(s);
    if (st) return st;
    const Species3 &sp = s->species[species];
    const int64_t n = sp.n;
    std::vector<uint32_t> key(n);
    std::vector<int32_t> pid(n);
    std::vector<double> L(3 * n), U(3 * n);
    const int b = s->pbuf;
    if ((st = download3(s, key.data(), s->d_key[b] + sp.offset, 4 * n))) return st;
    if ((st = download3(s, pid.data(), s->d_pid[b] + sp.offset, 4 * n))) return st;
    for (int c = 0; c < 3; ++c) {
        const size_t off = (c * s->p_cap + sp.offset) * s->rb();
        if ((st = download_reals3(s, &L[c * n], s->d_lam[b] + off, n))) return st;
        if ((st = download_reals3(s, &U[c * n], s->d_u[b] + off, n))) return st;
    }
    std::vector<std::pair<int32_t, int64_t>> live;
    live.reserve(n);
    for (int64_t i = 0; i < n; ++i)
        if (key[i] != kLost) live.push_back({pid[i], i});
    std::sort(live.begin(), live.end());
    if (n_out) *n_out = int64_t(live.size());
    if (!tet && !slot && !lam && !u && !id) return FETD_OK;
    if (capacity < int64_t(live.size())) return s->fail(FETD_E_ARG, "capacity too small");
    for (size_t j = 0; j < live.size(); ++j) {
        const int64_t i = live[j].second;
        if (tet) tet[j] = int32_t(key[i] & kTetMask);
        if (slot) slot[j] = int8_t(key[i] >> 30);
        for (int c = 0; c < 3; ++c) {
            if (lam) lam[3 * j + c] = L[c * n + i];
            if (u) u[3 * j + c] = U[c * n + i];
        }
        if (id) id[j] = live[j].first;
    }
    return FETD_OK;
}

fetd_status fetd3_diagnostics(fetd3_sim *s, fetd3_diag *out)
{
    if (!s || !out) return FETD_E_ARG;
    DeviceGuard3 g(s->device);
    std::memset(out, 0, sizeof *out);
    unsigned long long c[4];
    fetd_status st = download3(s, c, s->d_counters, sizeof c);
    if (st) return st;
    out->error_code = c[2] ? ((c[2] & 1) ? 1 : 2) : 0;
    out->step = s->step;
    out->n_segments = int64_t(c[0]);
    out->n_lost = int64_t(c[1]);
    out->n_nodes = s->nn;
    out->n_edges = s->ne;
    out->n_faces = s->nf;
    out->n_tets = s->nt;
    out->spai_frobenius = s->spai_fro;
    if (!s->have_baseline && (st = take_baseline3(s))) return st;
    if ((st = compute_charge3(s)) || (st = compute_divd3(s))) return st;
    std::vector<double> q(s->nn), dv(s->nn), e(s->ne), d(s->ne), b(s->nf), divb(s->nt);
    if ((st = download3(s, q.data(), s->d_q, 8 * q.size()))) return st;
    if ((st = download3(s, dv.data(), s->d_divd, 8 * dv.size()))) return st;
    if ((st = download3(s, e.data(), s->d_e, 8 * e.size()))) return st;
    if ((st = download3(s, d.data(), s->d_d, 8 * d.size()))) return st;
    if ((st = download3(s, b.data(), s->d_b, 8 * b.size()))) return st;
    hipError_t he = launch3_divb(s->stream, s->nt, s->d_tet_face, s->d_fout, s->d_b, s->d_divb);
    if (he != hipSuccess) return s->hip_fail(he, "divb");
    if ((st = download3(s, divb.data(), s->d_divb, 8 * divb.size()))) return st;
    double qm = 0, gm = 0;
    for (int n = 0; n < s->nn; ++n) {
        qm = std::max(qm, std::max(std::fabs(q[n]), std::fabs(s->q0[n])));
        if (s->node_free[n])
            gm = std::max(gm, std::fabs((dv[n] - s->divd0[n]) - (q[n] - s->q0[n])));
    }
    out->gauss_rel = qm > 0 ? gm / qm : gm;
    double bm = 0, dbm = 0;
    for (double v : b) bm = std::max(bm, std::fabs(v));
    for (double v : divb) dbm = std::max(dbm, std::fabs(v));
    out->divb_rel = bm > 0 ? dbm / bm : dbm;
    double we = 0;
    for (int i = 0; i < s->ne; ++i) we += e[i] * d[i];
    out->W_E = 0.5 * we;
    double wb = 0;
    for (int f = 0; f < s->nf; ++f) {
        double acc = 0;
        for (int j = s->mnu.ptr[f]; j < s->mnu.ptr[f + 1]; ++j) acc += s->mnu.val[j] * b[s->mnu.col[j]];
        wb += b[f] * acc;
    }
    out->W_B = 0.5 * wb;
    int64_t alive = 0;
    double wk = 0;
    for (const Species3 &sp : s->species) {
        if (sp.n == 0) continue;
        std::vector<uint32_t> key(sp.n);
        std::vector<double> U(3 * sp.n);
        if ((st = download3(s, key.data(), s->d_key[s->pbuf] + sp.offset, 4 * sp.n))) return st;
        for (int cc = 0; cc < 3; ++cc)
            if ((st = download_reals3(s, &U[cc * sp.n],
                                      s->d_u[s->pbuf] + (cc * s->p_cap + sp.offset) * s->rb(),
                                      sp.n)))
                return st;
        for (int64_t i = 0; i < sp.n; ++i) {
            if (key[i] == kLost) continue;
            ++alive;
            const double uu = U[i] * U[i] + U[sp.n + i] * U[sp.n + i] + U[2 * sp.n + i] * U[2 * sp.n + i];
            wk += sp.w * sp.m * s->c * s->c * (std::sqrt(1.0 + uu / (s->c * s->c)) - 1.0);
        }
    }
    out->n_alive = alive;
    out->W_kin = wk;
    return FETD_OK;
}

fetd_status fetd3_profile(fetd3_sim *s, int32_t enable)
{
    return fetd3_profile_mask(s, enable ? 0x1F : 0, 1);
}

fetd_status fetd3_profile_mask(fetd3_sim *s, int32_t stage_mask, int32_t every)
{
    if (!s || every < 1) return FETD_E_ARG;
    DeviceGuard3 g(s->device);
    s->resolve_timers();
    s->profile_mask = uint32_t(stage_mask) & 0x1Fu;
    s->profile_every = every;
    for (double &v : s->stage_ms) v = 0;
    s->particle_launches = 0;
    return FETD_OK;
}

fetd_status fetd3_stage_times(fetd3_sim *s, double *ms, int64_t *launches)
{
    if (!s || !ms) return FETD_E_ARG;
    DeviceGuard3 g(s->device);
    s->resolve_timers();
    for (int k = 0; k < 5; ++k) ms[k] = s->stage_ms[k];
    if (launches) *launches = s->particle_launches;
    return FETD_OK;
}

const char *fetd3_last_error(const fetd3_sim *s) { return s ? s->err.c_str() : g_err3.c_str(); }

void fetd3_destroy(fetd3_sim *s)
{
    if (!s) return;
    {
        DeviceGuard3 g(s->device);
        if (s->stream) (void)hipStreamSynchronize(s->stream);
        for (void *p : s->allocs) (void)hipFree(p);
        s->allocs.clear();
        if (s->h_alive) (void)hipHostFree(s->h_alive);
        for (hipEvent_t e : s->all_events) (void)hipEventDestroy(e);
        if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    }
    delete s;
}

}  // extern "C"
