// Host runtime of the FETD-PIC library: mesh tables, Hodge operators, the
// sparse approximate inverse, device state and the C-ABI entry points
// declared in include/fetdpic.h.
//
// Method: arXiv:1707.04333 (Na, Moon, Omelchenko, Teixeira), Sec. II.
#include "fetdpic.h"
#include "fetd_internal.h"
#include "fetd_sparse.h"
#include "stage_events.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

using namespace fetd;

static_assert(FETD_MAX_SPECIES_PARTICLES == kMaxSpeciesParticles, "particle limit");
static_assert(FETD_MAX_TRIS == kMaxTris, "mesh limit");

fetd_timing::Pending &fetd_timing::pending()
{
    thread_local Pending p;
    return p;
}

namespace {

thread_local std::string g_last_error;

struct Species {
    double q = 0, m = 0, w = 0;
    int64_t n_loaded = 0;  // ids 0..n_loaded-1
    int64_t n = 0;         // slots in use (alive + lost-but-not-yet-dropped)
    int64_t offset = 0;    // first slot in the particle arrays
    int64_t bc_offset = 0; // first per-tile counter slot (pairs) of the species
};

// Tiles of n particles at ppt particles per thread, and per-tile slots
// reserved per species (for the smallest tile a run may use).
int64_t tiles_of(int64_t n, int ppt = kPPT)
{
    return (n + int64_t(kBlock) * ppt - 1) / (int64_t(kBlock) * ppt);
}
int64_t slots_of(int64_t n) { return tiles_of(n, kMinPPT); }

}  // namespace

struct fetd_sim {
    // options
    int precision = FETD_FP64;
    double dt = 0, eps0 = 0, mu0 = 0, c = 0;
    int spai_level = 1;
    int device = 0;
    hipStream_t stream = nullptr;
    fetd_alloc_fn alloc_cb = nullptr;
    fetd_free_fn free_cb = nullptr;
    void *alloc_user = nullptr;
    int cap = 64;
    int resort_every = 20;
    double period[2] = {0, 0};

    // mesh (host)
    int nn = 0, nf = 0, ne = 0, n_free_e = 0, n_free_n = 0;
    std::vector<int32_t> tri_node, tri_edge, tri_nbr, edge_lo, edge_hi;
    std::vector<int8_t> tri_sign, tri_nbrk;
    std::vector<double> vxy, grad, area;
    std::vector<int32_t> edge_f;  // [2 ne]
    std::vector<int8_t> edge_s;   // [2 ne]
    std::vector<uint8_t> edge_free, node_free;
    std::vector<uint8_t> node_gauss;  // free and not touching a lossy edge
    // Device edge numbering: order of first appearance along the triangle
    // order (edges of nearby triangles get nearby ids).  Host tables and the
    // C-ABI use the canonical (low, high) lexicographic numbering.
    std::vector<int32_t> edev;       // canonical -> device id
    std::vector<int32_t> ecan;       // device id -> canonical
    std::vector<uint32_t> tri_ebase; // device edges first met before triangle f
    Csr meps, mt;
    double spai_fro = 0;

    // device: mesh
    int4 *d_tri_edge = nullptr, *d_tri_nbr = nullptr, *d_tri_node = nullptr, *d_edge_face = nullptr;
    int2 *d_edge_nodes = nullptr;
    uint32_t *d_tri_ebase = nullptr;
    double *d_grad64 = nullptr, *d_vxy64 = nullptr, *d_mu_area = nullptr, *d_two_area = nullptr;
    float *d_grad32 = nullptr, *d_vxy32 = nullptr;
    int32_t *d_sl_ptr = nullptr, *d_sl_w = nullptr, *d_sl_col = nullptr;
    void *d_sl_val = nullptr;  // FP64, or FP32 in the FP32-field mode
    // device: fields
    void *d_b = nullptr, *d_h = nullptr, *d_e = nullptr;  // field type (FP64 or FP32)
    double *d_d = nullptr;
    double *d_cur = nullptr;       // current accumulator of the step in progress
    double *d_cur_last = nullptr;  // current of the last completed step
    unsigned long long *d_fx = nullptr;  // deterministic mode: fixed-point current limbs [3 ne]
    bool deterministic = false;
    void *d_rec = nullptr;
    double *d_bz_ext = nullptr, *d_e_ext = nullptr, *d_damp = nullptr, *d_damp_b = nullptr;
    // uniaxial PML: rows (device edge ids), kappa, rows of the normal and
    // tangential parts of [*eps], auxiliary fluxes, and psi - phi per edge
    int pml_n = 0;
    int32_t *d_pml_rows = nullptr, *d_pn_ptr = nullptr, *d_pn_col = nullptr;
    int32_t *d_pt_ptr = nullptr, *d_pt_col = nullptr;
    double *d_pml_kappa = nullptr, *d_pn_val = nullptr, *d_pt_val = nullptr;
    double *d_pml_psi = nullptr, *d_pml_phi = nullptr, *d_pml_x = nullptr;
    bool has_affine = false;
    double e_scale = 1.0;  // multiplier of the applied edge field
    double affine[6] = {0, 0, 0, 0, 0, 0};
    // device: particles
    std::vector<Species> species;
    int64_t p_cap = 0;
    uint32_t *d_key[2] = {nullptr, nullptr};
    void *d_lam[2] = {nullptr, nullptr};
    void *d_u[2] = {nullptr, nullptr};
    int32_t *d_pid[2] = {nullptr, nullptr};
    int pbuf = 0;
    // device: sort and diagnostics scratch
    int32_t *d_counts = nullptr, *d_offsets = nullptr, *d_block_sums = nullptr;
    unsigned long long *d_counters = nullptr;
    unsigned long long *d_block_counts = nullptr;
    uint32_t *d_tile_home = nullptr;  // per tile, same slots as d_block_counts
    int ppt = kPPT;                   // particles per thread of the particle launches
    int xcap = 0;                     // crossing record: pieces kept per particle (0 = off)
    int32_t *d_xcount = nullptr, *d_xtris = nullptr;  // [p_cap], [p_cap * xcap]
    int scan = 64;                    // lanes per group of the first-piece current scan
    int defer = 0;                    // FP32 particles: deferred exits
    int64_t block_count_cap = 0;  // blocks covered by d_block_counts
    double *d_q = nullptr, *d_divd = nullptr, *d_partial = nullptr;
    // field probes
    int64_t probe_n = 0, probe_max = 0, probe_samples = 0;
    int32_t probe_every = 1, probe_in_window = 0;
    int32_t *d_probe_tri = nullptr;
    double *d_probe_lam = nullptr, *d_probe_acc = nullptr, *d_probe_buf = nullptr;
    static constexpr int kPartial = 1024;

    // state
    int64_t step = 0;
    int64_t steps_since_sort = 0;
    uint64_t desc_gen = 0;  // bumped when a buffer or value a batch descriptor holds changes
    bool have_baseline = false;
    std::vector<double> q0, divd0, q_last;
    int64_t q_last_step = -1;
    int64_t device_bytes = 0;
    std::string err;
    // stage timing
    uint32_t profile_mask = 0;  // bit k: stage k is timed
    int64_t profile_every = 1;  // on steps that are multiples of this
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timed[FETD_N_STAGES];
    std::vector<hipEvent_t> event_pool;
    hipEvent_t take_event()
    {
        hipEvent_t ev = nullptr;
        if (!event_pool.empty()) {
            ev = event_pool.back();
            event_pool.pop_back();
        } else if (hipEventCreate(&ev) != hipSuccess) {
            ev = nullptr;
        }
        return ev;
    }
    // Times a stage when timing is on.  The step stages (0-3) hand their
    // two events to the stage's kernel launches, which carry them in their
    // own dispatches; the sort (4) records them around its launches.
    struct Timer {
        fetd_sim *s;
        int stage;
        hipEvent_t a = nullptr, b = nullptr;
        Timer(fetd_sim *s_, int st) : s(s_), stage(st)
        {
            if (!(s->profile_mask >> stage & 1u) || s->step % s->profile_every != 0) return;
            a = s->take_event();
            b = a ? s->take_event() : nullptr;
            if (!b) {
                release();
                return;
            }
            if (stage == 4) {
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
        ~Timer()
        {
            if (!a) return;
            bool ok;
            if (stage == 4) {
                ok = hipEventRecord(b, s->stream) == hipSuccess;
            } else {
                ok = fetd_timing::pending().start == nullptr;  // a kernel took the events
                fetd_timing::pending() = {};
            }
            if (ok) s->timed[stage].push_back({a, b});
            else release();
        }
    };

    // ---------------------------------------------------------------
    fetd_status fail(fetd_status st, const std::string &msg)
    {
        err = msg;
        g_last_error = msg;
        return st;
    }
    fetd_status hip_fail(hipError_t e, const char *what)
    {
        return fail(FETD_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    }
    bool dev_alloc(void **p, size_t bytes)
    {
        if (bytes == 0) bytes = 16;
        if (alloc_cb) {
            *p = alloc_cb(bytes, alloc_user);
            if (!*p) return false;
        } else if (hipMalloc(p, bytes) != hipSuccess) {
            *p = nullptr;
            return false;
        }
        device_bytes += int64_t(bytes);
        allocs.push_back({*p, bytes});
        return true;
    }
    void dev_free(void *p)
    {
        if (!p) return;
        for (size_t i = 0; i < allocs.size(); ++i) {
            if (allocs[i].first == p) {
                device_bytes -= int64_t(allocs[i].second);
                allocs[i] = allocs.back();
                allocs.pop_back();
                break;
            }
        }
        if (free_cb) free_cb(p, alloc_user);
        else (void)hipFree(p);
    }
    std::vector<std::pair<void *, size_t>> allocs;

    // particle state in FP32 (both mixed modes); field state in FP32 (FETD_MIXED)
    bool fp32() const { return precision != FETD_FP64; }
    bool field32() const { return precision == FETD_MIXED; }
    size_t real_bytes() const { return fp32() ? 4 : 8; }
    size_t field_bytes() const { return field32() ? 4 : 8; }
};

namespace {

// ---------------------------------------------------------------------
// Mesh topology and geometry (Sec. II.A: incidence C, S; dual C~ = C^T).
// ---------------------------------------------------------------------
fetd_status build_topology(fetd_sim *s, const fetd_mesh_desc *md)
{
#pragma clang fp contract(off)
    const int nf = md->n_tris, nn = md->n_nodes;
    s->nf = nf;
    s->nn = nn;
    s->tri_node.assign(md->tri_nodes, md->tri_nodes + 3 * size_t(nf));
    for (int i = 0; i < 3 * nf; ++i)
        if (s->tri_node[i] < 0 || s->tri_node[i] >= nn)
            return s->fail(FETD_E_MESH, "triangle node id out of range");
    // vertex coordinates (image-consistent on periodic meshes)
    s->vxy.resize(6 * size_t(nf));
    for (int f = 0; f < nf; ++f)
        for (int k = 0; k < 3; ++k) {
            const int nd = s->tri_node[3 * f + k];
            double x = md->node_xy[2 * nd], y = md->node_xy[2 * nd + 1];
            if (md->tri_shift && md->period) {
                x = x + double(md->tri_shift[6 * f + 2 * k]) * md->period[0];
                y = y + double(md->tri_shift[6 * f + 2 * k + 1]) * md->period[1];
            }
            s->vxy[6 * f + 2 * k] = x;
            s->vxy[6 * f + 2 * k + 1] = y;
        }
    // area and grad lambda_k = perp(x_b - x_a) / 2A, perp(x, y) = (-y, x)
    s->area.resize(nf);
    s->grad.resize(6 * size_t(nf));
    for (int f = 0; f < nf; ++f) {
        const double *v = &s->vxy[6 * f];
        const double a2 = (v[2] - v[0]) * (v[5] - v[1]) - (v[4] - v[0]) * (v[3] - v[1]);
        if (!(a2 > 0)) return s->fail(FETD_E_MESH, "triangle " + std::to_string(f) +
                                                        " is not counter-clockwise");
        s->area[f] = 0.5 * a2;
        for (int k = 0; k < 3; ++k) {
            const int ia = (k + 1) % 3, ib = (k + 2) % 3;
            s->grad[6 * f + 2 * k] = -(v[2 * ib + 1] - v[2 * ia + 1]) / a2;
            s->grad[6 * f + 2 * k + 1] = (v[2 * ib] - v[2 * ia]) / a2;
        }
    }
    // edges: (low, high) node pairs in lexicographic order
    struct Occ {
        uint64_t key;
        int32_t fk;
    };
    std::vector<Occ> occ(3 * size_t(nf));
    for (int f = 0; f < nf; ++f)
        for (int k = 0; k < 3; ++k) {
            const int a = s->tri_node[3 * f + (k + 1) % 3], b = s->tri_node[3 * f + (k + 2) % 3];
            if (a == b) return s->fail(FETD_E_MESH, "degenerate edge");
            const uint64_t lo = uint64_t(std::min(a, b)), hi = uint64_t(std::max(a, b));
            occ[3 * f + k] = {(lo << 32) | hi, 3 * f + k};
        }
    std::sort(occ.begin(), occ.end(), [](const Occ &x, const Occ &y) {
        return x.key != y.key ? x.key < y.key : x.fk < y.fk;
    });
    s->tri_edge.assign(3 * size_t(nf), -1);
    s->tri_sign.assign(3 * size_t(nf), 0);
    s->tri_nbr.assign(3 * size_t(nf), -1);
    s->tri_nbrk.assign(3 * size_t(nf), -1);
    s->edge_lo.clear();
    s->edge_hi.clear();
    s->edge_f.clear();
    s->edge_s.clear();
    size_t i = 0;
    while (i < occ.size()) {
        size_t j = i;
        while (j < occ.size() && occ[j].key == occ[i].key) ++j;
        if (j - i > 2) return s->fail(FETD_E_MESH, "an edge has more than two triangles");
        const int ed = int(s->edge_lo.size());
        s->edge_lo.push_back(int32_t(occ[i].key >> 32));
        s->edge_hi.push_back(int32_t(occ[i].key & 0xffffffffu));
        int32_t ff[2] = {-1, -1};
        int8_t ss[2] = {0, 0};
        for (size_t t = i; t < j; ++t) {
            const int fk = occ[t].fk, f = fk / 3, k = fk % 3;
            const int a = s->tri_node[3 * f + (k + 1) % 3], b = s->tri_node[3 * f + (k + 2) % 3];
            s->tri_edge[fk] = ed;
            s->tri_sign[fk] = a < b ? 1 : -1;
            ff[t - i] = f;
            ss[t - i] = s->tri_sign[fk];
        }
        if (j - i == 2) {
            const int fa = occ[i].fk, fb = occ[i + 1].fk;
            s->tri_nbr[fa] = fb / 3;
            s->tri_nbrk[fa] = int8_t(fb % 3);
            s->tri_nbr[fb] = fa / 3;
            s->tri_nbrk[fb] = int8_t(fa % 3);
        }
        s->edge_f.push_back(ff[0]);
        s->edge_f.push_back(ff[1]);
        s->edge_s.push_back(ss[0]);
        s->edge_s.push_back(ss[1]);
        i = j;
    }
    s->ne = int(s->edge_lo.size());
    s->edge_free.assign(s->ne, 0);
    s->node_free.assign(nn, 1);
    s->n_free_e = 0;
    for (int e = 0; e < s->ne; ++e) {
        if (s->edge_f[2 * e + 1] >= 0) {
            s->edge_free[e] = 1;
            ++s->n_free_e;
        } else {
            s->node_free[s->edge_lo[e]] = 0;
            s->node_free[s->edge_hi[e]] = 0;
        }
    }
    s->n_free_n = 0;
    for (int n = 0; n < nn; ++n) s->n_free_n += s->node_free[n];
    s->edev.assign(s->ne, -1);
    s->ecan.assign(s->ne, -1);
    s->tri_ebase.assign(nf, 0);
    int next = 0;
    for (int f = 0; f < nf; ++f) {
        s->tri_ebase[f] = uint32_t(next);
        for (int k = 0; k < 3; ++k) {
            const int ed = s->tri_edge[3 * f + k];
            if (s->edev[ed] < 0) {
                s->edev[ed] = next;
                s->ecan[next] = ed;
                ++next;
            }
        }
    }
    s->node_gauss = s->node_free;
    return FETD_OK;
}

// [*eps]_ij = eps0 int W1_i . W1_j over the mesh (Sec. II.A), free edges.
void assemble_hodge_eps(fetd_sim *s)
{
    const int ne = s->ne;
    std::vector<std::vector<std::pair<int, double>>> rows(ne);
    for (int f = 0; f < s->nf; ++f) {
        const double *g = &s->grad[6 * f];
        const double A = s->area[f];
        auto gd = [&](int p, int q) { return g[2 * p] * g[2 * q] + g[2 * p + 1] * g[2 * q + 1]; };
        auto mass = [&](int p, int q) { return A * (p == q ? 2.0 : 1.0) / 12.0; };
        for (int k = 0; k < 3; ++k) {
            const int ek = s->tri_edge[3 * f + k];
            if (!s->edge_free[ek]) continue;
            const int a = (k + 1) % 3, b = (k + 2) % 3;
            for (int l = 0; l < 3; ++l) {
                const int el = s->tri_edge[3 * f + l];
                if (!s->edge_free[el]) continue;
                const int cc = (l + 1) % 3, dd = (l + 2) % 3;
                // int (l_a G_b - l_b G_a).(l_c G_d - l_d G_c)
                const double v = gd(b, dd) * mass(a, cc) - gd(b, cc) * mass(a, dd) -
                                 gd(a, dd) * mass(b, cc) + gd(a, cc) * mass(b, dd);
                rows[ek].push_back({el, s->eps0 * double(s->tri_sign[3 * f + k]) *
                                            double(s->tri_sign[3 * f + l]) * v});
            }
        }
    }
    Csr &M = s->meps;
    M.ptr.assign(ne + 1, 0);
    M.col.clear();
    M.val.clear();
    for (int e = 0; e < ne; ++e) {
        auto &r = rows[e];
        std::sort(r.begin(), r.end(),
                  [](const std::pair<int, double> &x, const std::pair<int, double> &y) {
                      return x.first < y.first;
                  });
        for (size_t t = 0; t < r.size(); ++t) {
            if (!M.col.empty() && int(M.col.size()) > M.ptr[e] && M.col.back() == r[t].first)
                M.val.back() += r[t].second;
            else {
                M.col.push_back(r[t].first);
                M.val.push_back(r[t].second);
            }
        }
        M.ptr[e + 1] = int32_t(M.col.size());
    }
}

fetd_status build_spai(fetd_sim *s, int level)
{
    if (!spai_build(s->meps, s->edge_free.data(), level, s->mt))
        return s->fail(FETD_E_MESH, "SPAI normal equations not positive definite");
    return FETD_OK;
}

// Exact inverse of the free block of [*eps] by dense Cholesky (small meshes).
fetd_status build_exact_inverse(fetd_sim *s)
{
    const int ne = s->ne;
    std::vector<int> fidx, pos(ne, -1);
    for (int e = 0; e < ne; ++e)
        if (s->edge_free[e]) {
            pos[e] = int(fidx.size());
            fidx.push_back(e);
        }
    const int n = int(fidx.size());
    if (n > 4096) return s->fail(FETD_E_ARG, "exact inverse limited to 4096 free edges");
    std::vector<double> L(size_t(n) * n, 0.0);
    for (int r = 0; r < n; ++r) {
        const int e = fidx[r];
        for (int q = s->meps.ptr[e]; q < s->meps.ptr[e + 1]; ++q)
            L[size_t(r) * n + pos[s->meps.col[q]]] = s->meps.val[q];
    }
    for (int j = 0; j < n; ++j) {
        double dgn = L[size_t(j) * n + j];
        for (int k = 0; k < j; ++k) dgn -= L[size_t(j) * n + k] * L[size_t(j) * n + k];
        if (!(dgn > 0)) return s->fail(FETD_E_MESH, "[*eps] not positive definite");
        dgn = std::sqrt(dgn);
        L[size_t(j) * n + j] = dgn;
        for (int i = j + 1; i < n; ++i) {
            double v = L[size_t(i) * n + j];
            for (int k = 0; k < j; ++k) v -= L[size_t(i) * n + k] * L[size_t(j) * n + k];
            L[size_t(i) * n + j] = v / dgn;
        }
    }
    std::vector<double> inv(size_t(n) * n, 0.0), col(n);
    for (int c = 0; c < n; ++c) {
        std::fill(col.begin(), col.end(), 0.0);
        col[c] = 1.0;
        for (int i = 0; i < n; ++i) {
            double v = col[i];
            for (int k = 0; k < i; ++k) v -= L[size_t(i) * n + k] * col[k];
            col[i] = v / L[size_t(i) * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double v = col[i];
            for (int k = i + 1; k < n; ++k) v -= L[size_t(k) * n + i] * col[k];
            col[i] = v / L[size_t(i) * n + i];
        }
        for (int i = 0; i < n; ++i) inv[size_t(i) * n + c] = col[i];
    }
    Csr &T = s->mt;
    T.ptr.assign(ne + 1, 0);
    T.col.clear();
    T.val.clear();
    for (int e = 0; e < ne; ++e) {
        if (pos[e] >= 0)
            for (int c = 0; c < n; ++c) {
                T.col.push_back(fidx[c]);
                T.val.push_back(0.5 * (inv[size_t(pos[e]) * n + c] + inv[size_t(c) * n + pos[e]]));
            }
        T.ptr[e + 1] = int32_t(T.col.size());
    }
    return FETD_OK;
}

template <typename T>
fetd_status upload(fetd_sim *s, T **dst, const T *src, size_t count)
{
    void *p = nullptr;
    if (!s->dev_alloc(&p, sizeof(T) * count))
        return s->fail(FETD_E_OOM, "device allocation failed");
    *dst = static_cast<T *>(p);
    if (count) {
        hipError_t e = hipMemcpyAsync(p, src, sizeof(T) * count, hipMemcpyHostToDevice, s->stream);
        if (e != hipSuccess) return s->hip_fail(e, "hipMemcpyAsync");
        e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return s->hip_fail(e, "hipStreamSynchronize");
    }
    return FETD_OK;
}

template <typename T>
fetd_status alloc_zero(fetd_sim *s, T **dst, size_t count)
{
    std::vector<T> z(count, T());
    return upload(s, dst, z.data(), count);
}

fetd_status upload_mesh(fetd_sim *s)
{
    const int nf = s->nf, ne = s->ne, nn = s->nn;
    std::vector<int4> te(nf), tn(nf), tno(nf);
    for (int f = 0; f < nf; ++f) {
        int sb = 0, kb = 0;
        for (int k = 0; k < 3; ++k) {
            if (s->tri_sign[3 * f + k] < 0) sb |= 1 << k;
            if (s->tri_nbrk[3 * f + k] >= 0) kb |= int(s->tri_nbrk[3 * f + k]) << (2 * k);
        }
        te[f] = make_int4(s->edev[s->tri_edge[3 * f]], s->edev[s->tri_edge[3 * f + 1]],
                          s->edev[s->tri_edge[3 * f + 2]], sb);
        tn[f] = make_int4(s->tri_nbr[3 * f], s->tri_nbr[3 * f + 1], s->tri_nbr[3 * f + 2], kb);
        tno[f] = make_int4(s->tri_node[3 * f], s->tri_node[3 * f + 1], s->tri_node[3 * f + 2], 0);
    }
    std::vector<int4> ef(ne);
    std::vector<int2> en(ne);
    for (int r = 0; r < ne; ++r) {
        const int e = s->ecan[r];
        ef[r] = make_int4(s->edge_f[2 * e], s->edge_f[2 * e + 1], s->edge_s[2 * e],
                          s->edge_s[2 * e + 1]);
        en[r] = make_int2(s->edge_lo[e], s->edge_hi[e]);
    }
    std::vector<float> g32(8 * size_t(nf), 0.f), v32(8 * size_t(nf), 0.f);
    std::vector<double> mua(nf), a2(nf);
    for (int f = 0; f < nf; ++f) {
        for (int k = 0; k < 6; ++k) {
            g32[8 * f + k] = float(s->grad[6 * f + k]);
            v32[8 * f + k] = float(s->vxy[6 * f + k]);
        }
        mua[f] = s->mu0 * s->area[f];
        a2[f] = 2.0 * s->area[f];
    }
    fetd_status st;
    if ((st = upload(s, &s->d_tri_edge, te.data(), nf))) return st;
    if ((st = upload(s, &s->d_tri_nbr, tn.data(), nf))) return st;
    if ((st = upload(s, &s->d_tri_node, tno.data(), nf))) return st;
    if ((st = upload(s, &s->d_edge_face, ef.data(), ne))) return st;
    if ((st = upload(s, &s->d_edge_nodes, en.data(), ne))) return st;
    if ((st = upload(s, &s->d_tri_ebase, s->tri_ebase.data(), s->tri_ebase.size()))) return st;
    if ((st = upload(s, &s->d_grad64, s->grad.data(), s->grad.size()))) return st;
    if ((st = upload(s, &s->d_vxy64, s->vxy.data(), s->vxy.size()))) return st;
    if ((st = upload(s, &s->d_grad32, g32.data(), g32.size()))) return st;
    if ((st = upload(s, &s->d_vxy32, v32.data(), v32.size()))) return st;
    if ((st = upload(s, &s->d_mu_area, mua.data(), mua.size()))) return st;
    if ((st = upload(s, &s->d_two_area, a2.data(), a2.size()))) return st;
    // SELL-64 of M~ in device edge order (wall rows are empty: e = 0 there)
    const int nsl = (ne + kSlice - 1) / kSlice;
    std::vector<int32_t> sp(nsl + 1, 0), sw(nsl, 0);
    for (int sl = 0; sl < nsl; ++sl) {
        int w = 0;
        for (int r = sl * kSlice; r < std::min(ne, (sl + 1) * kSlice); ++r)
            w = std::max(w, s->mt.ptr[s->ecan[r] + 1] - s->mt.ptr[s->ecan[r]]);
        sw[sl] = w;
        sp[sl + 1] = sp[sl] + w * kSlice;
    }
    std::vector<int32_t> scol(std::max(1, sp[nsl]), 0);
    std::vector<double> sval(std::max(1, sp[nsl]), 0.0);
    for (int sl = 0; sl < nsl; ++sl)
        for (int ln = 0; ln < kSlice; ++ln) {
            const int r = sl * kSlice + ln;
            for (int j = 0; j < sw[sl]; ++j) {
                const int q = sp[sl] + j * kSlice + ln;
                const int rr = std::min(r, ne - 1);
                const int rc = s->ecan[rr];
                if (r < ne && s->mt.ptr[rc] + j < s->mt.ptr[rc + 1]) {
                    scol[q] = s->edev[s->mt.col[s->mt.ptr[rc] + j]];
                    sval[q] = s->mt.val[s->mt.ptr[rc] + j];
                } else {
                    scol[q] = rr;
                    sval[q] = 0.0;
                }
            }
        }
    if ((st = upload(s, &s->d_sl_ptr, sp.data(), sp.size()))) return st;
    if ((st = upload(s, &s->d_sl_w, sw.data(), sw.size()))) return st;
    if ((st = upload(s, &s->d_sl_col, scol.data(), scol.size()))) return st;
    if (s->field32()) {
        std::vector<float> sv32(sval.begin(), sval.end());
        float *p32 = nullptr;
        if ((st = upload(s, &p32, sv32.data(), sv32.size()))) return st;
        s->d_sl_val = p32;
    } else {
        double *p64 = nullptr;
        if ((st = upload(s, &p64, sval.data(), sval.size()))) return st;
        s->d_sl_val = p64;
    }
    // fields (e, b, h in the field type; d and the currents in FP64)
    const size_t fb = s->field_bytes();
    for (void **fld : {&s->d_b, &s->d_h}) {
        char *p = nullptr;
        std::vector<char> z(fb * size_t(nf), 0);
        if ((st = upload(s, &p, z.data(), z.size()))) return st;
        *fld = p;
    }
    {
        char *p = nullptr;
        std::vector<char> z(fb * size_t(ne), 0);
        if ((st = upload(s, &p, z.data(), z.size()))) return st;
        s->d_e = p;
    }
    if ((st = alloc_zero(s, &s->d_d, ne))) return st;
    if ((st = alloc_zero(s, &s->d_cur, ne))) return st;
    if ((st = alloc_zero(s, &s->d_cur_last, ne))) return st;
    if (s->deterministic && (st = alloc_zero(s, &s->d_fx, 3 * size_t(ne)))) return st;
    void *rec = nullptr;
    if (!s->dev_alloc(&rec, 32 * size_t(nf)))
        return s->fail(FETD_E_OOM, "device allocation failed");
    s->d_rec = rec;
    if ((st = alloc_zero(s, &s->d_counts, size_t(nf) + 1))) return st;
    if ((st = alloc_zero(s, &s->d_offsets, size_t(nf) + 1))) return st;
    if ((st = alloc_zero(s, &s->d_block_sums, size_t(nf) / 1024 + 8))) return st;
    std::vector<unsigned long long> ctr = {0, 0, 0, std::numeric_limits<unsigned long long>::max()};
    if ((st = upload(s, &s->d_counters, ctr.data(), ctr.size()))) return st;
    if ((st = alloc_zero(s, &s->d_q, size_t(nn)))) return st;
    if ((st = alloc_zero(s, &s->d_divd, size_t(nn)))) return st;
    if ((st = alloc_zero(s, &s->d_partial, size_t(fetd_sim::kPartial)))) return st;
    return FETD_OK;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

fetd_status check_device_errors(fetd_sim *s)
{
    unsigned long long ctr[4];
    hipError_t e = hipMemcpyAsync(ctr, s->d_counters, sizeof ctr, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "device execution");
    if (ctr[2]) {
        return s->fail(FETD_E_TRACK, std::string(ctr[2] & 1 ? "crossing cap exceeded" :
                                                              "non-finite momentum") +
                                         " (first particle id " + std::to_string(ctr[3]) + ")");
    }
    return FETD_OK;
}

fetd_status download(fetd_sim *s, void *dst, const void *src, size_t bytes);

// Edge arrays cross the C-ABI in canonical order and live on the device in
// device order.
fetd_status download_edges(fetd_sim *s, double *dst, const double *d_src)
{
    std::vector<double> tmp(size_t(s->ne));
    if (fetd_status st = download(s, tmp.data(), d_src, 8 * tmp.size())) return st;
    for (int e = 0; e < s->ne; ++e) dst[e] = tmp[s->edev[e]];
    return FETD_OK;
}

fetd_status upload_edges(fetd_sim *s, double **d_dst, const double *src)
{
    std::vector<double> tmp(size_t(s->ne));
    for (int r = 0; r < s->ne; ++r) tmp[r] = src[s->ecan[r]];
    if (!*d_dst) return upload(s, d_dst, tmp.data(), tmp.size());
    hipError_t e = hipMemcpyAsync(*d_dst, tmp.data(), 8 * tmp.size(), hipMemcpyHostToDevice,
                                  s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "edge upload");
    return FETD_OK;
}

fetd_status grow_block_counts(fetd_sim *s, int64_t extra)
{
    // per-tile counter pairs: one region per species, the new one appended
    int64_t used = 0;
    for (const Species &sp : s->species) used = std::max(used, sp.bc_offset + slots_of(sp.n));
    const int64_t need = used + slots_of(extra) + 1;
    if (need > s->block_count_cap) {
        std::vector<unsigned long long> old(2 * size_t(need), 0ull);
        std::vector<uint32_t> home(size_t(need), 0u);
        if (s->block_count_cap > 0) {
            fetd_status st = download(s, old.data(), s->d_block_counts, 16 * size_t(s->block_count_cap));
            if (!st) st = download(s, home.data(), s->d_tile_home, 4 * size_t(s->block_count_cap));
            if (st) return st;
        }
        s->dev_free(s->d_block_counts);
        s->d_block_counts = nullptr;
        s->dev_free(s->d_tile_home);
        s->d_tile_home = nullptr;
        fetd_status st = upload(s, &s->d_block_counts, old.data(), old.size());
        if (!st) st = upload(s, &s->d_tile_home, home.data(), home.size());
        if (st) return st;
        s->block_count_cap = need;
    }
    return FETD_OK;
}

fetd_status grow_particles(fetd_sim *s, int64_t extra)
{
    if (fetd_status st = grow_block_counts(s, extra)) return st;
    const int64_t used = s->species.empty() ? 0 :
        s->species.back().offset + s->species.back().n;
    const int64_t need = used + extra;
    if (need <= s->p_cap) return FETD_OK;
    const size_t rb = s->real_bytes();
    int64_t ncap = std::max<int64_t>(need, 1024);
    uint32_t *key[2];
    void *lam[2], *u[2];
    int32_t *pid[2];
    for (int b = 0; b < 2; ++b) {
        void *p;
        if (!s->dev_alloc(&p, sizeof(uint32_t) * ncap)) return s->fail(FETD_E_OOM, "particles");
        key[b] = static_cast<uint32_t *>(p);
        if (!s->dev_alloc(&lam[b], 2 * rb * ncap)) return s->fail(FETD_E_OOM, "particles");
        if (!s->dev_alloc(&u[b], 2 * rb * ncap)) return s->fail(FETD_E_OOM, "particles");
        if (!s->dev_alloc(&p, sizeof(int32_t) * ncap)) return s->fail(FETD_E_OOM, "particles");
        pid[b] = static_cast<int32_t *>(p);
    }
    if (used > 0) {
        const int cb = s->pbuf;
        hipError_t e = hipMemcpyAsync(key[0], s->d_key[cb], sizeof(uint32_t) * used,
                                      hipMemcpyDeviceToDevice, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(lam[0], s->d_lam[cb], 2 * rb * used, hipMemcpyDeviceToDevice, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(u[0], s->d_u[cb], 2 * rb * used, hipMemcpyDeviceToDevice, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(pid[0], s->d_pid[cb], sizeof(int32_t) * used, hipMemcpyDeviceToDevice,
                               s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return s->hip_fail(e, "particle copy");
    }
    for (int b = 0; b < 2; ++b) {
        s->dev_free(s->d_key[b]);
        s->dev_free(s->d_lam[b]);
        s->dev_free(s->d_u[b]);
        s->dev_free(s->d_pid[b]);
        s->d_key[b] = key[b];
        s->d_lam[b] = lam[b];
        s->d_u[b] = u[b];
        s->d_pid[b] = pid[b];
    }
    s->pbuf = 0;
    s->p_cap = ncap;
    if (s->xcap > 0) {
        s->dev_free(s->d_xcount);
        s->dev_free(s->d_xtris);
        s->d_xcount = s->d_xtris = nullptr;
        fetd_status st = alloc_zero(s, &s->d_xcount, size_t(ncap));
        if (!st) st = alloc_zero(s, &s->d_xtris, size_t(ncap) * size_t(s->xcap));
        if (st) return st;
        ++s->desc_gen;
    }
    return FETD_OK;
}

fetd_status sort_all(fetd_sim *s, hipStream_t stream)
{
    const int cb = s->pbuf, ob = 1 - s->pbuf;
    const size_t rb = s->real_bytes();
    for (const Species &sp : s->species) {
        if (sp.n == 0) continue;
        SortArgs a;
        a.n = sp.n;
        a.nf = s->nf;
        a.key_in = s->d_key[cb] + sp.offset;
        a.lam_in = static_cast<char *>(s->d_lam[cb]) + 2 * rb * sp.offset;
        a.u_in = static_cast<char *>(s->d_u[cb]) + 2 * rb * sp.offset;
        a.pid_in = s->d_pid[cb] + sp.offset;
        a.key_out = s->d_key[ob] + sp.offset;
        a.lam_out = static_cast<char *>(s->d_lam[ob]) + 2 * rb * sp.offset;
        a.u_out = static_cast<char *>(s->d_u[ob]) + 2 * rb * sp.offset;
        a.pid_out = s->d_pid[ob] + sp.offset;
        a.counts = s->d_counts;
        a.offsets = s->d_offsets;
        a.block_sums = s->d_block_sums;
        a.elem_bytes = int(2 * rb);
        a.tile_home = s->d_tile_home + sp.bc_offset;
        a.tile = int64_t(s->ppt) * kBlock;
        // launch_sort writes the lost key into the slots past the live count
        hipError_t e = launch_sort(stream, a);
        if (e != hipSuccess) return s->hip_fail(e, "sort");
    }
    s->pbuf = ob;
    s->steps_since_sort = 0;
    return FETD_OK;
}

// Lanes per group of the particle kernel's first-piece current scan.
fetd_status set_defer(fetd_sim *s, int on)
{
    if (on != 0 && on != 1) return s->fail(FETD_E_ARG, "defer_exits must be 0 or 1");
    s->defer = on;
    return FETD_OK;
}

fetd_status set_scan(fetd_sim *s, int lanes)
{
    if (!valid_scan(lanes)) return s->fail(FETD_E_ARG, "scan_lanes must be 8, 16 or 64");
    if (lanes != s->scan) {
        s->scan = lanes;
        ++s->desc_gen;  // a batch holding this run rebuilds its descriptors
    }
    return FETD_OK;
}

// Switch the single-run particle launches to ppt particles per thread and
// recompute every tile's home triangle for the new tiling from the current
// particle order, on the simulation's stream (no allocation).
fetd_status set_ppt(fetd_sim *s, int ppt)
{
    if (!valid_ppt(ppt)) return s->fail(FETD_E_ARG, "invalid tile size");
    if (ppt == s->ppt) return FETD_OK;
    s->ppt = ppt;
    ++s->desc_gen;  // a batch holding this run rebuilds its tile list
    for (const Species &sp : s->species) {
        if (sp.n == 0) continue;
        hipError_t e = launch_tile_home(s->stream, sp.n, s->d_key[s->pbuf] + sp.offset,
                                        s->d_tile_home + sp.bc_offset, int64_t(ppt) * kBlock);
        if (e != hipSuccess) return s->hip_fail(e, "tile homes");
    }
    return FETD_OK;
}

fetd_status compute_charge(fetd_sim *s)
{
    hipError_t e = hipMemsetAsync(s->d_q, 0, sizeof(double) * size_t(s->nn), s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "charge");
    const size_t rb = s->real_bytes();
    for (const Species &sp : s->species) {
        e = launch_charge(s->stream, sp.n, s->d_key[s->pbuf] + sp.offset,
                          static_cast<char *>(s->d_lam[s->pbuf]) + 2 * rb * sp.offset, s->fp32(),
                          s->d_tri_node, sp.q * sp.w, s->d_q);
        if (e != hipSuccess) return s->hip_fail(e, "charge");
    }
    return FETD_OK;
}

fetd_status compute_divd(fetd_sim *s)
{
    hipError_t e = hipMemsetAsync(s->d_divd, 0, sizeof(double) * size_t(s->nn), s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "divd");
    e = launch_divd(s->stream, s->ne, s->d_edge_nodes, s->d_d, s->d_divd);
    if (e != hipSuccess) return s->hip_fail(e, "divd");
    return FETD_OK;
}

fetd_status download(fetd_sim *s, void *dst, const void *src, size_t bytes)
{
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "download");
    return FETD_OK;
}

fetd_status take_baseline(fetd_sim *s)
{
    fetd_status st;
    if ((st = compute_charge(s)) || (st = compute_divd(s))) return st;
    s->q0.resize(s->nn);
    s->divd0.resize(s->nn);
    if ((st = download(s, s->q0.data(), s->d_q, sizeof(double) * s->nn))) return st;
    if ((st = download(s, s->divd0.data(), s->d_divd, sizeof(double) * s->nn))) return st;
    s->have_baseline = true;
    return FETD_OK;
}

// Exponent E of the deterministic accumulator: a current contribution is
// sigma (Q/dt) w_k with |w_k| <= 1 up to rounding, so every contribution of
// the step is below 2^E in magnitude.
int fx_exponent(const fetd_sim *s)
{
    double m = 0.0;
    for (const Species &sp : s->species) m = std::max(m, std::fabs(sp.q * sp.w / s->dt));
    return m > 0.0 ? std::ilogb(m) + 2 : 0;
}

MeshView mesh_view(const fetd_sim *s)
{
    MeshView mv;
    mv.tri_edge = s->d_tri_edge;
    mv.tri_nbr = s->d_tri_nbr;
    mv.grad64 = s->d_grad64;
    mv.grad32 = s->d_grad32;
    mv.vxy64 = s->d_vxy64;
    mv.vxy32 = s->d_vxy32;
    mv.tri_ebase = s->d_tri_ebase;
    return mv;
}

FieldDesc field_desc(const fetd_sim *s)
{
    FieldDesc d{};
    d.nf = s->nf;
    d.ne = s->ne;
    d.rec_fp32 = s->fp32() ? 1 : 0;
    d.field32 = s->field32() ? 1 : 0;
    d.tri_edge = s->d_tri_edge;
    d.e = s->d_e;
    d.e_ext = s->d_e_ext;
    d.e_scale = s->e_scale;
    d.b = s->d_b;
    d.damp_b = s->d_damp_b;
    d.h = s->d_h;
    d.mu_area = s->d_mu_area;
    d.two_area = s->d_two_area;
    d.bz_ext = s->d_bz_ext;
    d.grad64 = s->d_grad64;
    d.rec = s->d_rec;
    d.dt = s->dt;
    d.edge_face = s->d_edge_face;
    d.cur = s->d_cur;
    d.cur_last = s->d_cur_last;
    d.d = s->d_d;
    d.damp = s->d_damp;
    d.fx = s->d_fx;
    d.fx_unscale = std::ldexp(1.0, fx_exponent(s) - 96);
    d.pml_n = s->pml_n;
    d.pml_rows = s->d_pml_rows;
    d.pml_kappa = s->d_pml_kappa;
    d.pn_ptr = s->d_pn_ptr;
    d.pn_col = s->d_pn_col;
    d.pn_val = s->d_pn_val;
    d.pt_ptr = s->d_pt_ptr;
    d.pt_col = s->d_pt_col;
    d.pt_val = s->d_pt_val;
    d.pml_psi = s->d_pml_psi;
    d.pml_phi = s->d_pml_phi;
    d.pml_x = s->pml_n > 0 ? s->d_pml_x : nullptr;
    d.sl_ptr = s->d_sl_ptr;
    d.sl_w = s->d_sl_w;
    d.sl_col = s->d_sl_col;
    d.sl_val = s->d_sl_val;
    d.e_out = s->d_e;
    return d;
}

StepArgs step_args(const fetd_sim *s, const Species &sp, int pbuf)
{
    const size_t rb = s->real_bytes();
    StepArgs a;
    a.n = sp.n;
    a.key = s->d_key[pbuf] + sp.offset;
    a.lam = static_cast<char *>(s->d_lam[pbuf]) + 2 * rb * sp.offset;
    a.u = static_cast<char *>(s->d_u[pbuf]) + 2 * rb * sp.offset;
    a.pid = s->d_pid[pbuf] + sp.offset;
    a.rec = s->d_rec;
    a.cur = s->d_cur;
    a.fx = s->d_fx;
    a.fx_scale = std::ldexp(1.0, 96 - fx_exponent(s));
    a.qdt = sp.q * sp.w / s->dt;
    a.alpha = sp.q * s->dt / (2.0 * sp.m);
    a.dt = s->dt;
    a.c = s->c;
    a.c2 = s->c * s->c;
    a.inv_c2 = 1.0 / (s->c * s->c);
    a.cap = s->cap;
    a.has_affine = s->has_affine ? 1 : 0;
    for (int k = 0; k < 6; ++k) a.aff[k] = s->affine[k];
    a.counters = s->d_counters;
    a.block_counts = s->d_block_counts + 2 * sp.bc_offset;
    a.tile_home = s->d_tile_home + sp.bc_offset;
    a.ppt = s->ppt;
    a.scan = s->scan;
    a.defer = s->defer;
    a.xcap = s->xcap;
    a.xcount = s->d_xcount ? s->d_xcount + sp.offset : nullptr;
    a.xtris = s->d_xtris ? s->d_xtris + sp.offset * s->xcap : nullptr;
    return a;
}

// A field array (e, b: the field type) to host doubles; edge arrays are
// permuted from device to canonical order.
fetd_status download_field(fetd_sim *s, double *dst, const void *src, int64_t n, bool edge)
{
    std::vector<double> tmp(static_cast<size_t>(n));
    if (s->field32()) {
        std::vector<float> f(static_cast<size_t>(n));
        if (fetd_status st = download(s, f.data(), src, 4 * size_t(n))) return st;
        for (int64_t i = 0; i < n; ++i) tmp[i] = double(f[i]);
    } else if (fetd_status st = download(s, tmp.data(), src, 8 * size_t(n))) {
        return st;
    }
    if (edge)
        for (int64_t e = 0; e < n; ++e) dst[e] = tmp[s->edev[e]];
    else
        std::copy(tmp.begin(), tmp.end(), dst);
    return FETD_OK;
}

// Release the uniaxial PML's device arrays (the layer's magnetic loss
// d_damp_b stays, shared with the absorber; its owner clears it).
void clear_pml(fetd_sim *s)
{
    for (void *p : {(void *)s->d_pml_rows, (void *)s->d_pn_ptr, (void *)s->d_pn_col,
                    (void *)s->d_pt_ptr, (void *)s->d_pt_col, (void *)s->d_pml_kappa,
                    (void *)s->d_pn_val, (void *)s->d_pt_val, (void *)s->d_pml_psi,
                    (void *)s->d_pml_phi, (void *)s->d_pml_x})
        s->dev_free(p);
    s->d_pml_rows = s->d_pn_ptr = s->d_pn_col = s->d_pt_ptr = s->d_pt_col = nullptr;
    s->d_pml_kappa = s->d_pn_val = s->d_pt_val = nullptr;
    s->d_pml_psi = s->d_pml_phi = s->d_pml_x = nullptr;
    s->pml_n = 0;
}

// Rows of the parts of [*eps] carried by the x (comp 0) or y (comp 1)
// component of the Whitney 1-forms, eps0 int W_i,c W_j,c (Sec. II.A), for
// the canonical edge rows listed; columns in increasing canonical order.
void hodge_part_rows(const fetd_sim *s, int comp, const std::vector<int> &rows,
                     std::vector<int32_t> &ptr, std::vector<int32_t> &col,
                     std::vector<double> &val)
{
    std::vector<int> slot(s->ne, -1);
    for (size_t k = 0; k < rows.size(); ++k) slot[rows[k]] = int(k);
    std::vector<std::vector<std::pair<int, double>>> acc(rows.size());
    for (int f = 0; f < s->nf; ++f) {
        const double *g = &s->grad[6 * f];
        const double A = s->area[f];
        auto gd = [&](int p, int q) { return g[2 * p + comp] * g[2 * q + comp]; };
        auto mass = [&](int p, int q) { return A * (p == q ? 2.0 : 1.0) / 12.0; };
        for (int k = 0; k < 3; ++k) {
            const int ek = s->tri_edge[3 * f + k];
            if (slot[ek] < 0 || !s->edge_free[ek]) continue;
            const int a = (k + 1) % 3, b = (k + 2) % 3;
            for (int l = 0; l < 3; ++l) {
                const int el = s->tri_edge[3 * f + l];
                if (!s->edge_free[el]) continue;
                const int cc = (l + 1) % 3, dd = (l + 2) % 3;
                const double v = gd(b, dd) * mass(a, cc) - gd(b, cc) * mass(a, dd) -
                                 gd(a, dd) * mass(b, cc) + gd(a, cc) * mass(b, dd);
                acc[slot[ek]].push_back({el, s->eps0 * double(s->tri_sign[3 * f + k]) *
                                                 double(s->tri_sign[3 * f + l]) * v});
            }
        }
    }
    ptr.assign(1, 0);
    col.clear();
    val.clear();
    for (auto &r : acc) {
        std::stable_sort(r.begin(), r.end(),
                         [](const std::pair<int, double> &x, const std::pair<int, double> &y) {
                             return x.first < y.first;
                         });
        for (size_t t = 0; t < r.size(); ++t) {
            if (int(col.size()) > ptr.back() && col.back() == s->edev[r[t].first])
                val.back() += r[t].second;
            else {
                col.push_back(s->edev[r[t].first]);
                val.push_back(r[t].second);
            }
        }
        ptr.push_back(int32_t(col.size()));
    }
}

}  // namespace

// =====================================================================
// C-ABI
// =====================================================================
extern "C" {

fetd_status fetd_mesh_create(const fetd_mesh_desc *mesh, const fetd_opts *opts, fetd_sim **out)
{
    if (!out) {
        g_last_error = "out is NULL";
        return FETD_E_ARG;
    }
    *out = nullptr;
    if (!mesh || !opts || !mesh->node_xy || !mesh->tri_nodes || mesh->n_nodes <= 0 ||
        mesh->n_tris <= 0) {
        g_last_error = "invalid mesh description";
        return FETD_E_ARG;
    }
    if (mesh->n_tris > FETD_MAX_TRIS) {
        g_last_error = "mesh has more than FETD_MAX_TRIS triangles";
        return FETD_E_ARG;
    }
    // c^2 within [1e-250, 1e250]: the FP64 pushers' division by c^2 is
    // correctly rounded on that range.
    if (!(opts->dt > 0) || !(opts->eps0 > 0) || !(opts->mu0 > 0) || !(opts->c > 0) ||
        !(opts->c * opts->c >= 1e-250 && opts->c * opts->c <= 1e250) ||
        (opts->precision != FETD_FP64 && opts->precision != FETD_MIXED &&
         opts->precision != FETD_MIXED_F64FIELD) ||
        opts->spai_level < -1 || opts->spai_level > 4) {
        g_last_error = "invalid options";
        return FETD_E_ARG;
    }
    fetd_sim *s = new (std::nothrow) fetd_sim();
    if (!s) {
        g_last_error = "out of host memory";
        return FETD_E_OOM;
    }
    s->precision = opts->precision;
    s->dt = opts->dt;
    s->eps0 = opts->eps0;
    s->mu0 = opts->mu0;
    s->c = opts->c;
    s->spai_level = opts->spai_level;
    s->device = opts->device;
    s->stream = static_cast<hipStream_t>(opts->stream);
    s->alloc_cb = opts->alloc;
    s->free_cb = opts->free;
    s->alloc_user = opts->alloc_user;
    s->cap = opts->crossing_cap > 0 ? opts->crossing_cap : 64;
    s->resort_every = opts->resort_every > 0 ? opts->resort_every : 20;
    s->deterministic = opts->deterministic != 0;
    s->xcap = opts->record_crossings;
    if (s->xcap < 0 || s->xcap > 64) {
        delete s;
        g_last_error = "record_crossings must be 0..64";
        return FETD_E_ARG;
    }
    if ((s->alloc_cb == nullptr) != (s->free_cb == nullptr)) {
        delete s;
        g_last_error = "alloc and free callbacks must be given together";
        return FETD_E_ARG;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || opts->device < 0 || opts->device >= ndev) {
        delete s;
        g_last_error = "no such HIP device";
        return FETD_E_HIP;
    }
    if (mesh->period && mesh->tri_shift) {
        s->period[0] = mesh->period[0];
        s->period[1] = mesh->period[1];
    }
    DeviceGuard g(s->device);
    fetd_status st = build_topology(s, mesh);
    if (st == FETD_OK) {
        assemble_hodge_eps(s);
        st = s->spai_level < 0 ? build_exact_inverse(s) : build_spai(s, s->spai_level);
    }
    if (st == FETD_OK) {
        s->spai_fro = spai_frobenius(s->meps, s->mt, s->edge_free.data(), s->n_free_e);
        st = upload_mesh(s);
    }
    if (st != FETD_OK) {
        g_last_error = s->err;
        fetd_destroy(s);
        return st;
    }
    *out = s;
    return FETD_OK;
}

void fetd_destroy(fetd_sim *s)
{
    if (!s) return;
    DeviceGuard g(s->device);
    (void)hipStreamSynchronize(s->stream);
    auto allocs = s->allocs;
    for (auto &a : allocs) s->dev_free(a.first);
    for (auto &v : s->timed)
        for (auto &p : v) {
            (void)hipEventDestroy(p.first);
            (void)hipEventDestroy(p.second);
        }
    for (auto ev : s->event_pool) (void)hipEventDestroy(ev);
    delete s;
}

const char *fetd_last_error(const fetd_sim *s)
{
    if (s) return s->err.c_str();
    return g_last_error.c_str();
}

fetd_status fetd_fields_set(fetd_sim *s, const double *bz_ext, const double *e_ext,
                            const double *e_affine)
{
    if (!s) return FETD_E_ARG;
    DeviceGuard g(s->device);
    ++s->desc_gen;
    fetd_status st;
    if (bz_ext) {
        if (!s->d_bz_ext && (st = alloc_zero(s, &s->d_bz_ext, s->nf))) return st;
        hipError_t e = hipMemcpyAsync(s->d_bz_ext, bz_ext, sizeof(double) * s->nf,
                                      hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return s->hip_fail(e, "fields_set");
    } else if (s->d_bz_ext) {
        s->dev_free(s->d_bz_ext);
        s->d_bz_ext = nullptr;
    }
    if (e_ext) {
        if ((st = upload_edges(s, &s->d_e_ext, e_ext))) return st;
    } else if (s->d_e_ext) {
        s->dev_free(s->d_e_ext);
        s->d_e_ext = nullptr;
    }
    s->has_affine = e_affine != nullptr;
    for (int k = 0; k < 6; ++k) s->affine[k] = e_affine ? e_affine[k] : 0.0;
    return FETD_OK;
}

fetd_status fetd_set_ext_scale(fetd_sim *s, double scale)
{
    if (!s) return FETD_E_ARG;
    if (!std::isfinite(scale)) return s->fail(FETD_E_ARG, "scale must be finite");
    s->e_scale = scale;
    ++s->desc_gen;
    return FETD_OK;
}

fetd_status fetd_set_absorber(fetd_sim *s, const double *sigma_tri)
{
    if (!s) return FETD_E_ARG;
    DeviceGuard g(s->device);
    if (sigma_tri)
        for (int f = 0; f < s->nf; ++f)
            if (!(sigma_tri[f] >= 0.0) || !std::isfinite(sigma_tri[f]))
                return s->fail(FETD_E_ARG, "conductivity must be finite and >= 0");
    if (hipError_t e = hipStreamSynchronize(s->stream)) return s->hip_fail(e, "set_absorber");
    clear_pml(s);
    s->node_gauss = s->node_free;
    ++s->desc_gen;
    if (!sigma_tri) {
        s->dev_free(s->d_damp);
        s->dev_free(s->d_damp_b);
        s->d_damp = s->d_damp_b = nullptr;
        return FETD_OK;
    }
    // Electric loss on edges (conductivity averaged over the edge's
    // triangles) and the matched magnetic loss sigma_m = sigma mu0 / eps0 on
    // triangles: both decay with the factor (1 - x) / (1 + x),
    // x = sigma dt / (2 eps0), so the layer's wave impedance stays that of
    // free space.
    auto factor = [s](double sg) {
        const double x = sg * s->dt / (2.0 * s->eps0);
        return sg > 0.0 ? (1.0 - x) / (1.0 + x) : 1.0;
    };
    std::vector<double> damp(s->ne, 1.0), damp_b(s->nf, 1.0);
    for (int e = 0; e < s->ne; ++e) {
        const int f0 = s->edge_f[2 * e], f1 = s->edge_f[2 * e + 1];
        double sg = sigma_tri[f0];
        if (f1 >= 0) sg = 0.5 * (sigma_tri[f0] + sigma_tri[f1]);
        if (sg > 0.0) {
            damp[e] = factor(sg);
            s->node_gauss[s->edge_lo[e]] = 0;
            s->node_gauss[s->edge_hi[e]] = 0;
        }
    }
    for (int f = 0; f < s->nf; ++f) damp_b[f] = factor(sigma_tri[f]);
    fetd_status st = upload_edges(s, &s->d_damp, damp.data());
    if (st) return st;
    if (!s->d_damp_b) return upload(s, &s->d_damp_b, damp_b.data(), damp_b.size());
    hipError_t e = hipMemcpyAsync(s->d_damp_b, damp_b.data(), 8 * damp_b.size(),
                                  hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "absorber upload");
    return FETD_OK;
}

fetd_status fetd_set_pml(fetd_sim *s, const double *sigma_tri, int32_t axis)
{
    if (!s) return FETD_E_ARG;
    if (axis != 0 && axis != 1) return s->fail(FETD_E_ARG, "axis must be 0 (x) or 1 (y)");
    DeviceGuard g(s->device);
    if (sigma_tri)
        for (int f = 0; f < s->nf; ++f)
            if (!(sigma_tri[f] >= 0.0) || !std::isfinite(sigma_tri[f]))
                return s->fail(FETD_E_ARG, "conductivity must be finite and >= 0");
    if (hipError_t e = hipStreamSynchronize(s->stream)) return s->hip_fail(e, "set_pml");
    clear_pml(s);
    s->dev_free(s->d_damp);
    s->dev_free(s->d_damp_b);
    s->d_damp = s->d_damp_b = nullptr;
    s->node_gauss = s->node_free;  // d is updated without loss: Gauss holds everywhere
    ++s->desc_gen;
    if (!sigma_tri) return FETD_OK;
    // the layer's rows: free edges whose conductivity (mean of their
    // triangles) is positive; kappa = sigma / eps0
    std::vector<int> rows;
    std::vector<int32_t> drows;
    std::vector<double> kappa;
    for (int r = 0; r < s->ne; ++r) {
        const int e = s->ecan[r];  // device order
        if (!s->edge_free[e]) continue;
        const int f0 = s->edge_f[2 * e], f1 = s->edge_f[2 * e + 1];
        const double sg = f1 >= 0 ? 0.5 * (sigma_tri[f0] + sigma_tri[f1]) : sigma_tri[f0];
        if (sg > 0.0) {
            rows.push_back(e);
            drows.push_back(r);
            kappa.push_back(sg / s->eps0);
        }
    }
    // matched magnetic loss on b (the stretched permeability mu0 s)
    std::vector<double> damp_b(s->nf, 1.0);
    for (int f = 0; f < s->nf; ++f) {
        const double x = sigma_tri[f] * s->dt / (2.0 * s->eps0);
        if (sigma_tri[f] > 0.0) damp_b[f] = (1.0 - x) / (1.0 + x);
    }
    fetd_status st = upload(s, &s->d_damp_b, damp_b.data(), damp_b.size());
    if (st || rows.empty()) return st;
    std::vector<int32_t> nptr, ncol, tptr, tcol;
    std::vector<double> nval, tval;
    hodge_part_rows(s, axis, rows, nptr, ncol, nval);
    hodge_part_rows(s, 1 - axis, rows, tptr, tcol, tval);
    const size_t n = rows.size();
    if ((st = upload(s, &s->d_pml_rows, drows.data(), n))) return st;
    if ((st = upload(s, &s->d_pml_kappa, kappa.data(), n))) return st;
    if ((st = upload(s, &s->d_pn_ptr, nptr.data(), nptr.size()))) return st;
    if ((st = upload(s, &s->d_pn_col, ncol.data(), ncol.size()))) return st;
    if ((st = upload(s, &s->d_pn_val, nval.data(), nval.size()))) return st;
    if ((st = upload(s, &s->d_pt_ptr, tptr.data(), tptr.size()))) return st;
    if ((st = upload(s, &s->d_pt_col, tcol.data(), tcol.size()))) return st;
    if ((st = upload(s, &s->d_pt_val, tval.data(), tval.size()))) return st;
    if ((st = alloc_zero(s, &s->d_pml_psi, n))) return st;
    if ((st = alloc_zero(s, &s->d_pml_phi, n))) return st;
    if ((st = alloc_zero(s, &s->d_pml_x, size_t(s->ne)))) return st;
    s->pml_n = int(n);
    return FETD_OK;
}

fetd_status fetd_fields_load(fetd_sim *s, const double *b, const double *d)
{
    if (!s) return FETD_E_ARG;
    DeviceGuard g(s->device);
    if (b)
        for (int f = 0; f < s->nf; ++f)
            if (!std::isfinite(b[f])) return s->fail(FETD_E_ARG, "b must be finite");
    if (d)
        for (int e = 0; e < s->ne; ++e)
            if (!std::isfinite(d[e])) return s->fail(FETD_E_ARG, "d must be finite");
    if (hipError_t e = hipStreamSynchronize(s->stream)) return s->hip_fail(e, "fields_load");
    // the PML's auxiliary fluxes restart from zero with the loaded state
    if (s->pml_n > 0) {
        hipError_t e = launch_fill_u32(s->stream, reinterpret_cast<uint32_t *>(s->d_pml_psi), 0u,
                                       2 * int64_t(s->pml_n));
        if (e == hipSuccess)
            e = launch_fill_u32(s->stream, reinterpret_cast<uint32_t *>(s->d_pml_phi), 0u,
                                2 * int64_t(s->pml_n));
        if (e == hipSuccess)
            e = launch_fill_u32(s->stream, reinterpret_cast<uint32_t *>(s->d_pml_x), 0u,
                                2 * int64_t(s->ne));
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return s->hip_fail(e, "fields_load pml");
    }
    if (b) {
        std::vector<float> b32;
        const void *src = b;
        if (s->field32()) {
            b32.assign(b, b + s->nf);
            src = b32.data();
        }
        hipError_t e = hipMemcpyAsync(s->d_b, src, s->field_bytes() * size_t(s->nf),
                                      hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return s->hip_fail(e, "b upload");
    }
    if (d) {
        // wall edges carry no degree of freedom
        std::vector<double> df(d, d + s->ne);
        for (int e = 0; e < s->ne; ++e)
            if (!s->edge_free[e]) df[e] = 0.0;
        fetd_status st = upload_edges(s, &s->d_d, df.data());
        if (st) return st;
        hipError_t e = launch_spmv(s->stream, field_desc(s));
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return s->hip_fail(e, "fields_load spmv");
    }
    // Gauss's law is accounted from this state on
    s->have_baseline = false;
    return FETD_OK;
}

fetd_status fetd_particles_load_bary(fetd_sim *s, double q, double m, double w, int64_t n,
                                     const int32_t *tri, const int8_t *slot, const double *lam,
                                     const double *u, int32_t *species_out)
{
    if (!s) return FETD_E_ARG;
    if (n > FETD_MAX_SPECIES_PARTICLES)
        return s->fail(FETD_E_ARG, "species has more than FETD_MAX_SPECIES_PARTICLES particles");
    if (n < 0 || (n > 0 && (!tri || !lam || !u)) || !(m > 0))
        return s->fail(FETD_E_ARG, "invalid particle arguments");
    DeviceGuard g(s->device);
    for (int64_t i = 0; i < n; ++i) {
        if (tri[i] < 0 || tri[i] >= s->nf) return s->fail(FETD_E_ARG, "triangle id out of range");
        if (slot && (slot[i] < 0 || slot[i] > 2)) return s->fail(FETD_E_ARG, "slot out of range");
    }
    ++s->desc_gen;
    fetd_status st = grow_particles(s, n);
    if (st) return st;
    Species sp;
    sp.q = q;
    sp.m = m;
    sp.w = w;
    sp.n_loaded = n;
    sp.n = n;
    sp.offset = s->species.empty() ? 0 : s->species.back().offset + s->species.back().n;
    sp.bc_offset = s->species.empty() ? 0 :
        s->species.back().bc_offset + slots_of(s->species.back().n);
    const size_t rb = s->real_bytes();
    std::vector<uint32_t> key(n);
    std::vector<int32_t> pid(n);
    std::vector<char> lb(2 * rb * n), ub(2 * rb * n);
    for (int64_t i = 0; i < n; ++i) {
        key[i] = uint32_t(tri[i]) | (uint32_t(slot ? slot[i] : 0) << 30);
        pid[i] = int32_t(i);
        if (s->fp32()) {
            float *lf = reinterpret_cast<float *>(lb.data()), *uf = reinterpret_cast<float *>(ub.data());
            lf[2 * i] = float(lam[2 * i]);
            lf[2 * i + 1] = float(lam[2 * i + 1]);
            uf[2 * i] = float(u[2 * i]);
            uf[2 * i + 1] = float(u[2 * i + 1]);
        } else {
            std::memcpy(lb.data() + 16 * i, lam + 2 * i, 16);
            std::memcpy(ub.data() + 16 * i, u + 2 * i, 16);
        }
    }
    const int cb = s->pbuf;
    hipError_t e = hipSuccess;
    if (n > 0) {
        e = hipMemcpyAsync(s->d_key[cb] + sp.offset, key.data(), 4 * n, hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(static_cast<char *>(s->d_lam[cb]) + 2 * rb * sp.offset, lb.data(),
                               2 * rb * n, hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(static_cast<char *>(s->d_u[cb]) + 2 * rb * sp.offset, ub.data(),
                               2 * rb * n, hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->d_pid[cb] + sp.offset, pid.data(), 4 * n, hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    }
    if (e != hipSuccess) return s->hip_fail(e, "particles_load");
    s->species.push_back(sp);
    if (species_out) *species_out = int32_t(s->species.size() - 1);
    s->have_baseline = false;
    // sorted order for the segmented deposit
    if (n > 0 && (st = sort_all(s, s->stream))) return st;
    return FETD_OK;
}

// Point location: for each point the lowest-id triangle containing it (on
// periodic axes, the point or an image one period away) and its barycentric
// pair (lambda_1, lambda_2).  `what` names the points in the error message.
fetd_status locate_points(fetd_sim *s, int64_t n, const double *xy, std::vector<int32_t> &tri,
                          std::vector<double> &lam, const char *what,
                          const int32_t *hint = nullptr)
{
#pragma clang fp contract(off)
    // uniform bucket grid over triangle bounding boxes
    double x0 = 1e300, y0 = 1e300, x1 = -1e300, y1 = -1e300;
    for (int f = 0; f < s->nf; ++f)
        for (int k = 0; k < 3; ++k) {
            x0 = std::min(x0, s->vxy[6 * f + 2 * k]);
            x1 = std::max(x1, s->vxy[6 * f + 2 * k]);
            y0 = std::min(y0, s->vxy[6 * f + 2 * k + 1]);
            y1 = std::max(y1, s->vxy[6 * f + 2 * k + 1]);
        }
    const int nb = std::max(1, int(std::sqrt(double(s->nf) / 2.0)));
    const double bx = (x1 - x0) / nb, by = (y1 - y0) / nb;
    std::vector<std::vector<int>> bucket(size_t(nb) * nb);
    for (int f = 0; f < s->nf; ++f) {
        double lx = 1e300, ly = 1e300, hx = -1e300, hy = -1e300;
        for (int k = 0; k < 3; ++k) {
            lx = std::min(lx, s->vxy[6 * f + 2 * k]);
            hx = std::max(hx, s->vxy[6 * f + 2 * k]);
            ly = std::min(ly, s->vxy[6 * f + 2 * k + 1]);
            hy = std::max(hy, s->vxy[6 * f + 2 * k + 1]);
        }
        const int i0 = std::clamp(int((lx - x0) / bx), 0, nb - 1), i1 = std::clamp(int((hx - x0) / bx), 0, nb - 1);
        const int j0 = std::clamp(int((ly - y0) / by), 0, nb - 1), j1 = std::clamp(int((hy - y0) / by), 0, nb - 1);
        for (int j = j0; j <= j1; ++j)
            for (int i = i0; i <= i1; ++i) bucket[size_t(j) * nb + i].push_back(f);
    }
    // the point and, on periodic axes, its images one period away (triangle
    // frames of a periodic mesh extend past the period cell)
    tri.assign(size_t(n), -1);
    lam.assign(2 * size_t(n), 0.0);
    const int mx = s->period[0] > 0 ? 1 : 0, my = s->period[1] > 0 ? 1 : 0;
    // barycentric pair of (qx, qy) in triangle f, true if inside or on it
    auto inside = [s](int f, double qx, double qy, double &l1, double &l2) {
        const double *v = &s->vxy[6 * f];
        const double den = (v[2] - v[0]) * (v[5] - v[1]) - (v[4] - v[0]) * (v[3] - v[1]);
        l1 = ((qx - v[0]) * (v[5] - v[1]) - (v[4] - v[0]) * (qy - v[1])) / den;
        l2 = ((v[2] - v[0]) * (qy - v[1]) - (qx - v[0]) * (v[3] - v[1])) / den;
        return l1 >= 0 && l2 >= 0 && l1 + l2 <= 1;
    };
    for (int64_t p = 0; p < n; ++p) {
        int best = -1;
        double bl1 = 0, bl2 = 0;
        if (hint && hint[p] >= 0 && hint[p] < s->nf) {
            for (int sx = -mx; sx <= mx && best < 0; ++sx)
                for (int sy = -my; sy <= my && best < 0; ++sy) {
                    double l1, l2;
                    if (inside(hint[p], xy[2 * p] + double(sx) * s->period[0],
                               xy[2 * p + 1] + double(sy) * s->period[1], l1, l2)) {
                        best = hint[p];
                        bl1 = l1;
                        bl2 = l2;
                    }
                }
            if (best >= 0) {
                tri[p] = best;
                lam[2 * p] = bl1;
                lam[2 * p + 1] = bl2;
                continue;
            }
        }
        for (int sx = -mx; sx <= mx; ++sx)
            for (int sy = -my; sy <= my; ++sy) {
                const double qx = xy[2 * p] + double(sx) * s->period[0];
                const double qy = xy[2 * p + 1] + double(sy) * s->period[1];
                if (qx < x0 || qx > x1 || qy < y0 || qy > y1) continue;
                const int bi = std::clamp(int((qx - x0) / bx), 0, nb - 1);
                const int bj = std::clamp(int((qy - y0) / by), 0, nb - 1);
                for (int f : bucket[size_t(bj) * nb + bi]) {
                    if (best >= 0 && f >= best) break;
                    double l1, l2;
                    if (inside(f, qx, qy, l1, l2)) {
                        best = f;
                        bl1 = l1;
                        bl2 = l2;
                        break;
                    }
                }
            }
        if (best < 0)
            return s->fail(FETD_E_ARG, std::string(what) + " " + std::to_string(p) +
                                           " is outside the mesh");
        tri[p] = best;
        lam[2 * p] = bl1;
        lam[2 * p + 1] = bl2;
    }
    return FETD_OK;
}

fetd_status fetd_particles_load(fetd_sim *s, double q, double m, double w, int64_t n,
                                const double *xy, const double *u, const int32_t *tri_hint,
                                int32_t *species_out)
{
    if (!s) return FETD_E_ARG;
    if (n > FETD_MAX_SPECIES_PARTICLES)
        return s->fail(FETD_E_ARG, "species has more than FETD_MAX_SPECIES_PARTICLES particles");
    if (n < 0 || (n > 0 && (!xy || !u))) return s->fail(FETD_E_ARG, "invalid particle arguments");
    std::vector<int32_t> tri;
    std::vector<double> lam;
    if (fetd_status st = locate_points(s, n, xy, tri, lam, "particle", tri_hint)) return st;
    return fetd_particles_load_bary(s, q, m, w, n, tri.data(), nullptr, lam.data(), u, species_out);
}

fetd_status fetd_sort(fetd_sim *s)
{
    if (!s) return FETD_E_ARG;
    DeviceGuard g(s->device);
    fetd_sim::Timer t(s, 4);
    return sort_all(s, s->stream);
}

fetd_status fetd_pic_step(fetd_sim *s, int32_t n_steps, int32_t pusher)
{
    if (!s) return FETD_E_ARG;
    if (n_steps < 0 || pusher < 0 || pusher > 3) return s->fail(FETD_E_ARG, "invalid step arguments");
    DeviceGuard g(s->device);
    fetd_status st;
    if (!s->have_baseline && (st = take_baseline(s))) return st;
    const MeshView mv = mesh_view(s);
    const FieldDesc fd = field_desc(s);
    for (int it = 0; it < n_steps; ++it) {
        if (s->steps_since_sort >= s->resort_every) {
            fetd_sim::Timer t(s, 4);
            if ((st = sort_all(s, s->stream))) return st;
        }
        hipError_t e;
        {
            fetd_sim::Timer t(s, 0);
            e = launch_faraday(s->stream, fd);
        }
        if (e != hipSuccess) return s->hip_fail(e, "faraday");
        for (const Species &sp : s->species) {
            const StepArgs a = step_args(s, sp, s->pbuf);
            fetd_sim::Timer t(s, 1);
            e = launch_particles(s->stream, mv, a, pusher, s->fp32());
            if (e != hipSuccess) return s->hip_fail(e, "particle step");
        }
        {
            fetd_sim::Timer t(s, 2);
            e = launch_ampere(s->stream, fd);
        }
        if (e != hipSuccess) return s->hip_fail(e, "ampere");
        {
            fetd_sim::Timer t(s, 3);
            if (s->pml_n > 0) e = launch_pml_aux(s->stream, fd);
            if (e == hipSuccess) e = launch_spmv(s->stream, fd);
        }
        if (e != hipSuccess) return s->hip_fail(e, "spmv");
        if (s->probe_n > 0 && s->probe_samples < s->probe_max) {
            const bool flush = ++s->probe_in_window == s->probe_every;
            double *out = flush ? s->d_probe_buf + 2 * s->probe_n * s->probe_samples : nullptr;
            e = launch_probe(s->stream, int(s->probe_n), s->d_probe_tri, s->d_probe_lam,
                             s->d_tri_edge, s->d_grad64, s->d_e, s->field32(), s->d_probe_acc,
                             out, 1.0 / double(s->probe_every));
            if (e != hipSuccess) return s->hip_fail(e, "probe");
            if (flush) {
                ++s->probe_samples;
                s->probe_in_window = 0;
            }
        }
        ++s->step;
        ++s->steps_since_sort;
    }
    return FETD_OK;
}

fetd_status fetd_probe_set(fetd_sim *s, int64_t n, const double *xy, int32_t every,
                           int64_t max_samples)
{
    if (!s) return FETD_E_ARG;
    DeviceGuard g(s->device);
    if (n < 0 || (n > 0 && (!xy || every < 1 || max_samples < 1)) || n > (int64_t(1) << 30))
        return s->fail(FETD_E_ARG, "invalid probe arguments");
    if (hipError_t e = hipStreamSynchronize(s->stream)) return s->hip_fail(e, "probe_set");
    for (void *p : {(void *)s->d_probe_tri, (void *)s->d_probe_lam, (void *)s->d_probe_acc,
                    (void *)s->d_probe_buf})
        s->dev_free(p);
    s->d_probe_tri = nullptr;
    s->d_probe_lam = s->d_probe_acc = s->d_probe_buf = nullptr;
    s->probe_n = s->probe_max = s->probe_samples = 0;
    s->probe_in_window = 0;
    if (n == 0) return FETD_OK;
    std::vector<int32_t> tri;
    std::vector<double> lam;
    if (fetd_status st = locate_points(s, n, xy, tri, lam, "probe")) return st;
    fetd_status st = upload(s, &s->d_probe_tri, tri.data(), tri.size());
    if (!st) st = upload(s, &s->d_probe_lam, lam.data(), lam.size());
    if (!st) st = alloc_zero(s, &s->d_probe_acc, 2 * size_t(n));
    if (st) return st;
    void *p = nullptr;
    if (!s->dev_alloc(&p, sizeof(double) * 2 * size_t(n) * size_t(max_samples)))
        return s->fail(FETD_E_OOM, "probe buffer");
    s->d_probe_buf = static_cast<double *>(p);
    s->probe_n = n;
    s->probe_max = max_samples;
    s->probe_every = every;
    return FETD_OK;
}

fetd_status fetd_probe_get(fetd_sim *s, double *dst, int64_t capacity_bytes, int64_t *n_samples)
{
    if (!s) return FETD_E_ARG;
    DeviceGuard g(s->device);
    if (n_samples) *n_samples = s->probe_samples;
    const size_t bytes = sizeof(double) * 2 * size_t(s->probe_n) * size_t(s->probe_samples);
    if (!dst || bytes == 0) return FETD_OK;
    if (capacity_bytes < int64_t(bytes)) return s->fail(FETD_E_ARG, "destination too small");
    return download(s, dst, s->d_probe_buf, bytes);
}

fetd_status fetd_sync(fetd_sim *s)
{
    if (!s) return FETD_E_ARG;
    DeviceGuard g(s->device);
    return check_device_errors(s);
}

fetd_status fetd_fields_get(fetd_sim *s, int32_t which, void *dst, int64_t capacity,
                            int64_t *written)
{
    if (!s) return FETD_E_ARG;
    DeviceGuard g(s->device);
    fetd_status st = check_device_errors(s);
    if (st) return st;
    const void *src = nullptr;
    size_t bytes = 0;
    bool host = false, edge = false, field = false;
    std::vector<int32_t> tmp;
    switch (which) {
    case FETD_FIELD_E: src = s->d_e; bytes = 8 * size_t(s->ne); edge = true; field = true; break;
    case FETD_FIELD_D: src = s->d_d; bytes = 8 * size_t(s->ne); edge = true; break;
    case FETD_FIELD_B: src = s->d_b; bytes = 8 * size_t(s->nf); field = true; break;
    case FETD_FIELD_J: src = s->d_cur_last; bytes = 8 * size_t(s->ne); edge = true; break;
    case FETD_FIELD_Q:
        if ((st = compute_charge(s))) return st;
        src = s->d_q;
        bytes = 8 * size_t(s->nn);
        break;
    case FETD_FIELD_DIVD:
        if ((st = compute_divd(s))) return st;
        src = s->d_divd;
        bytes = 8 * size_t(s->nn);
        break;
    case FETD_FIELD_SPAI_PTR: src = s->mt.ptr.data(); bytes = 4 * s->mt.ptr.size(); host = true; break;
    case FETD_FIELD_SPAI_COL: src = s->mt.col.data(); bytes = 4 * s->mt.col.size(); host = true; break;
    case FETD_FIELD_SPAI_VAL: src = s->mt.val.data(); bytes = 8 * s->mt.val.size(); host = true; break;
    case FETD_FIELD_EDGES:
        tmp.resize(2 * size_t(s->ne));
        for (int e = 0; e < s->ne; ++e) {
            tmp[2 * e] = s->edge_lo[e];
            tmp[2 * e + 1] = s->edge_hi[e];
        }
        src = tmp.data();
        bytes = 4 * tmp.size();
        host = true;
        break;
    case FETD_FIELD_TRI_EDGE: src = s->tri_edge.data(); bytes = 4 * s->tri_edge.size(); host = true; break;
    default: return s->fail(FETD_E_ARG, "unknown field selector");
    }
    if (written) *written = int64_t(bytes);
    if (!dst) return FETD_OK;
    if (capacity < int64_t(bytes)) return s->fail(FETD_E_ARG, "destination too small");
    if (host) {
        std::memcpy(dst, src, bytes);
        return FETD_OK;
    }
    if (field)
        return download_field(s, static_cast<double *>(dst), src, int64_t(bytes / 8), edge);
    if (edge) return download_edges(s, static_cast<double *>(dst), static_cast<const double *>(src));
    return download(s, dst, src, bytes);
}

fetd_status fetd_particles_get(fetd_sim *s, int32_t species, int64_t capacity, int32_t *tri,
                               int8_t *slot, double *lam, double *u, int64_t *id, int64_t *n_out)
{
    if (!s) return FETD_E_ARG;
    if (species < 0 || species >= int32_t(s->species.size()))
        return s->fail(FETD_E_ARG, "no such species");
    DeviceGuard g(s->device);
    fetd_status st = check_device_errors(s);
    if (st) return st;
    const Species &sp = s->species[species];
    const size_t rb = s->real_bytes();
    std::vector<uint32_t> key(sp.n);
    std::vector<int32_t> pid(sp.n);
    std::vector<char> lb(2 * rb * sp.n), ub(2 * rb * sp.n);
    if (sp.n) {
        if ((st = download(s, key.data(), s->d_key[s->pbuf] + sp.offset, 4 * sp.n))) return st;
        if ((st = download(s, pid.data(), s->d_pid[s->pbuf] + sp.offset, 4 * sp.n))) return st;
        if ((st = download(s, lb.data(), static_cast<char *>(s->d_lam[s->pbuf]) + 2 * rb * sp.offset,
                           2 * rb * sp.n)))
            return st;
        if ((st = download(s, ub.data(), static_cast<char *>(s->d_u[s->pbuf]) + 2 * rb * sp.offset,
                           2 * rb * sp.n)))
            return st;
    }
    std::vector<std::pair<int32_t, int64_t>> order;
    order.reserve(sp.n);
    for (int64_t i = 0; i < sp.n; ++i)
        if (key[i] != kLost) order.push_back({pid[i], i});
    std::sort(order.begin(), order.end());
    if (n_out) *n_out = int64_t(order.size());
    if (capacity < int64_t(order.size())) return s->fail(FETD_E_ARG, "capacity too small");
    for (size_t o = 0; o < order.size(); ++o) {
        const int64_t i = order[o].second;
        if (tri) tri[o] = int32_t(key[i] & kTriMask);
        if (slot) slot[o] = int8_t(key[i] >> 30);
        if (id) id[o] = order[o].first;
        for (int c = 0; c < 2; ++c) {
            if (s->fp32()) {
                if (lam) lam[2 * o + c] = double(reinterpret_cast<float *>(lb.data())[2 * i + c]);
                if (u) u[2 * o + c] = double(reinterpret_cast<float *>(ub.data())[2 * i + c]);
            } else {
                if (lam) lam[2 * o + c] = reinterpret_cast<double *>(lb.data())[2 * i + c];
                if (u) u[2 * o + c] = reinterpret_cast<double *>(ub.data())[2 * i + c];
            }
        }
    }
    return FETD_OK;
}

fetd_status fetd_crossings_get(fetd_sim *s, int32_t species, int64_t capacity, int32_t *count,
                               int32_t *tris, int64_t *n_out)
{
    if (!s) return FETD_E_ARG;
    if (s->xcap <= 0) return s->fail(FETD_E_STATE, "record_crossings is off");
    if (species < 0 || species >= int32_t(s->species.size()))
        return s->fail(FETD_E_ARG, "no such species");
    DeviceGuard g(s->device);
    fetd_status st = check_device_errors(s);
    if (st) return st;
    const Species &sp = s->species[species];
    const int K = s->xcap;
    std::vector<uint32_t> key(sp.n);
    std::vector<int32_t> pid(sp.n), cnt(sp.n), seq(size_t(sp.n) * K);
    if (sp.n) {
        if ((st = download(s, key.data(), s->d_key[s->pbuf] + sp.offset, 4 * sp.n))) return st;
        if ((st = download(s, pid.data(), s->d_pid[s->pbuf] + sp.offset, 4 * sp.n))) return st;
        if ((st = download(s, cnt.data(), s->d_xcount + sp.offset, 4 * sp.n))) return st;
        if ((st = download(s, seq.data(), s->d_xtris + sp.offset * K, 4 * size_t(sp.n) * K)))
            return st;
    }
    std::vector<std::pair<int32_t, int64_t>> order;
    order.reserve(sp.n);
    for (int64_t i = 0; i < sp.n; ++i)
        if (key[i] != kLost) order.push_back({pid[i], i});
    std::sort(order.begin(), order.end());
    if (n_out) *n_out = int64_t(order.size());
    if (capacity < int64_t(order.size())) return s->fail(FETD_E_ARG, "capacity too small");
    for (size_t o = 0; o < order.size(); ++o) {
        const int64_t i = order[o].second;
        if (count) count[o] = cnt[i];
        if (tris)
            for (int k = 0; k < K; ++k)
                tris[o * K + k] = k < cnt[i] ? seq[size_t(i) * K + k] : -1;
    }
    return FETD_OK;
}

fetd_status fetd_diagnostics(fetd_sim *s, fetd_diag *out)
{
    if (!s || !out) return FETD_E_ARG;
    DeviceGuard g(s->device);
    std::memset(out, 0, sizeof *out);
    unsigned long long ctr[4];
    fetd_status st = download(s, ctr, s->d_counters, sizeof ctr);
    if (st) return st;
    out->error_code = int32_t(ctr[2] & 1 ? 1 : (ctr[2] & 2 ? 2 : 0));
    out->error_particle = ctr[2] ? int64_t(ctr[3]) : -1;
    if (!s->have_baseline && (st = take_baseline(s))) return st;
    if ((st = compute_charge(s)) || (st = compute_divd(s))) return st;
    const int nn = s->nn, ne = s->ne;
    std::vector<double> q(nn), dv(nn), e(ne), d(ne), b(s->nf), jl(ne);
    if ((st = download(s, q.data(), s->d_q, 8 * size_t(nn)))) return st;
    if ((st = download(s, dv.data(), s->d_divd, 8 * size_t(nn)))) return st;
    if ((st = download_field(s, e.data(), s->d_e, ne, true))) return st;
    if ((st = download_edges(s, d.data(), s->d_d))) return st;
    if ((st = download_field(s, b.data(), s->d_b, s->nf, false))) return st;
    if ((st = download_edges(s, jl.data(), s->d_cur_last))) return st;
    double gmax = 0, qmax = 0;
    for (int n = 0; n < nn; ++n) {
        qmax = std::max(qmax, std::max(std::fabs(q[n]), std::fabs(s->q0[n])));
        if (!s->node_gauss[n]) continue;
        gmax = std::max(gmax, std::fabs((dv[n] - s->divd0[n]) - (q[n] - s->q0[n])));
    }
    out->gauss_abs = gmax;
    out->gauss_rel = qmax > 0 ? gmax / qmax : 0.0;
    out->dce_abs = -1;
    out->dce_rel = -1;
    if (s->q_last_step >= 0 && s->q_last_step + 1 == s->step) {
        std::vector<double> divj(nn, 0.0);
        for (int ed = 0; ed < ne; ++ed) {
            divj[s->edge_lo[ed]] += jl[ed];
            divj[s->edge_hi[ed]] -= jl[ed];
        }
        double dm = 0, qm = 0;
        for (int n = 0; n < nn; ++n) {
            qm = std::max(qm, std::max(std::fabs(q[n]), std::fabs(s->q_last[n])));
            if (!s->node_gauss[n]) continue;
            dm = std::max(dm, std::fabs((q[n] - s->q_last[n]) + s->dt * divj[n]));
        }
        out->dce_abs = dm;
        out->dce_rel = qm > 0 ? dm / qm : 0.0;
    }
    s->q_last = q;
    s->q_last_step = s->step;
    double we = 0, wb = 0;
    for (int ed = 0; ed < ne; ++ed) we += e[ed] * d[ed];
    for (int f = 0; f < s->nf; ++f) wb += b[f] * b[f] / (s->mu0 * s->area[f]);
    out->W_E = 0.5 * we;
    out->W_B = 0.5 * wb;
    double wk = 0;
    const size_t rb = s->real_bytes();
    std::vector<double> part(fetd_sim::kPartial);
    int64_t alive = 0;
    for (const Species &sp : s->species) {
        hipError_t err = hipMemsetAsync(s->d_partial, 0, 8 * fetd_sim::kPartial, s->stream);
        if (err != hipSuccess) return s->hip_fail(err, "kinetic");
        err = launch_kinetic(s->stream, sp.n, s->d_key[s->pbuf] + sp.offset,
                             static_cast<char *>(s->d_u[s->pbuf]) + 2 * rb * sp.offset, s->fp32(),
                             1.0 / (s->c * s->c), s->d_partial, fetd_sim::kPartial);
        if (err != hipSuccess) return s->hip_fail(err, "kinetic");
        if ((st = download(s, part.data(), s->d_partial, 8 * fetd_sim::kPartial))) return st;
        double acc = 0;
        for (double v : part) acc += v;
        wk += sp.w * sp.m * s->c * s->c * acc;
        alive += sp.n_loaded;
    }
    out->W_kin = wk;
    out->step = s->step;
    unsigned long long nseg = 0, nlost = 0;
    if (s->block_count_cap > 0) {
        std::vector<unsigned long long> bc(2 * size_t(s->block_count_cap));
        if ((st = download(s, bc.data(), s->d_block_counts, 8 * bc.size()))) return st;
        for (size_t b = 0; b < bc.size(); b += 2) {
            nseg += bc[b];
            nlost += bc[b + 1];
        }
    }
    out->n_lost = int64_t(nlost);
    out->n_alive = alive - out->n_lost;
    out->n_segments = int64_t(nseg);
    if (ctr[2]) {
        s->err = std::string("device error flag ") + std::to_string(ctr[2]);
        return FETD_E_TRACK;
    }
    return FETD_OK;
}

fetd_status fetd_profile(fetd_sim *s, int32_t enable)
{
    return fetd_profile_mask(s, enable ? (1 << FETD_N_STAGES) - 1 : 0, 1);
}

fetd_status fetd_profile_mask(fetd_sim *s, int32_t stage_mask, int32_t every)
{
    if (!s || every < 1) return FETD_E_ARG;
    DeviceGuard g(s->device);
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "profile");
    for (auto &v : s->timed) {
        for (auto &p : v) {
            s->event_pool.push_back(p.first);
            s->event_pool.push_back(p.second);
        }
        v.clear();
    }
    s->profile_mask = uint32_t(stage_mask) & ((1u << FETD_N_STAGES) - 1);
    s->profile_every = every;
    return FETD_OK;
}

fetd_status fetd_stage_times(fetd_sim *s, double *ms, int64_t *launches)
{
    if (!s || !ms || !launches) return FETD_E_ARG;
    DeviceGuard g(s->device);
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "stage_times");
    for (int k = 0; k < FETD_N_STAGES; ++k) {
        double tot = 0.0;
        for (auto &p : s->timed[k]) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, p.first, p.second) == hipSuccess) tot += double(t);
        }
        ms[k] = tot;
        launches[k] = int64_t(s->timed[k].size());
    }
    return FETD_OK;
}

fetd_status fetd_set_resort(fetd_sim *s, int32_t every)
{
    if (!s || every < 1) return FETD_E_ARG;
    s->resort_every = every;
    return FETD_OK;
}

// Particle-stage milliseconds of each of the last `steps` steps (the
// events of stage 1, one launch per species and step), from a run of
// `steps` steps with re-sorting off.
static fetd_status timed_particle_steps(fetd_sim *s, int32_t pusher, int32_t steps,
                                        std::vector<double> &tp)
{
    const int nsp = int(std::count_if(s->species.begin(), s->species.end(),
                                      [](const Species &x) { return x.n > 0; }));
    tp.assign(size_t(steps), 0.0);
    fetd_status st;
    if ((st = fetd_profile_mask(s, (1 << 1) | (1 << 4), 1))) return st;
    if ((st = fetd_pic_step(s, steps, pusher))) return st;
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "autotune");
    const auto &ev = s->timed[1];
    for (size_t k = 0; k < ev.size(); ++k) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, ev[k].first, ev[k].second) == hipSuccess && nsp > 0)
            tp[std::min<size_t>(k / nsp, size_t(steps) - 1)] += double(t);
    }
    return FETD_OK;
}

fetd_status fetd_autotune(fetd_sim *s, int32_t pusher, int32_t trial_steps, fetd_tuning *out)
{
    if (!s || trial_steps < 2 || pusher < 0 || pusher > 3) return FETD_E_ARG;
    DeviceGuard g(s->device);
    fetd_status st;
    const int32_t was_mask = int32_t(s->profile_mask);
    const int32_t was_every = int32_t(s->profile_every);
    const int saved = s->resort_every;
    s->resort_every = std::numeric_limits<int>::max();
    std::vector<double> tp;
    const int short_steps = std::min<int32_t>(trial_steps, 20);
    if (out) {
        for (double &c : out->resort_cost_ms) c = -1.0;
        for (double &c : out->tile_cost_ms) c = -1.0;
        for (double &c : out->scan_cost_ms) c = -1.0;
        for (double &c : out->defer_cost_ms) c = -1.0;
    }
    // Mean particle-stage ms per step over short_steps steps from a fresh sort.
    auto trial = [&](double &cost) -> fetd_status {
        fetd_status e;
        if ((e = sort_all(s, s->stream))) return e;
        if ((e = timed_particle_steps(s, pusher, short_steps, tp))) return e;
        double sum = 0.0;
        for (double t : tp) sum += t;
        cost = sum / short_steps;
        return FETD_OK;
    };

    // 1. Tile (the current one first, so a tie keeps it).
    {
        int order[kNumPPT] = {s->ppt};
        for (int k = 0, j = 1; k < kNumPPT; ++k)
            if (kPPTChoices[k] != s->ppt) order[j++] = kPPTChoices[k];
        int best = s->ppt;
        double best_cost = std::numeric_limits<double>::max();
        for (int c : order) {
            double cost = 0.0;
            if ((st = set_ppt(s, c)) || (st = trial(cost))) return st;
            for (int k = 0; k < kNumPPT; ++k)
                if (kPPTChoices[k] == c && out) out->tile_cost_ms[k] = cost;
            if (cost < best_cost) {
                best_cost = cost;
                best = c;
            }
        }
        if ((st = set_ppt(s, best))) return st;
    }
    // 2. Scan group width, with that tile.
    {
        int order[3] = {s->scan, 0, 0};
        for (int k = 0, j = 1; k < 3; ++k)
            if (kScanChoices[k] != s->scan) order[j++] = kScanChoices[k];
        int best = s->scan;
        double best_cost = std::numeric_limits<double>::max();
        for (int c : order) {
            double cost = 0.0;
            if ((st = set_scan(s, c)) || (st = trial(cost))) return st;
            for (int k = 0; k < 3; ++k)
                if (kScanChoices[k] == c && out) out->scan_cost_ms[k] = cost;
            if (cost < best_cost) {
                best_cost = cost;
                best = c;
            }
        }
        if ((st = set_scan(s, best))) return st;
    }
    // 3. Deferred exits (FP32 particles; FP64 always defers), with that tile
    //    and width.
    if (s->fp32()) {
        const int first = s->defer;
        int best = first;
        double best_cost = std::numeric_limits<double>::max();
        for (int c : {first, 1 - first}) {
            double cost = 0.0;
            if ((st = set_defer(s, c)) || (st = trial(cost))) return st;
            if (out) out->defer_cost_ms[c] = cost;
            if (cost < best_cost) {
                best_cost = cost;
                best = c;
            }
        }
        if ((st = set_defer(s, best))) return st;
    }


    // 4. Re-sort cadence: one timed sort, then the particle stage of every
    //    step as the order decays.
    if ((st = fetd_profile_mask(s, (1 << 1) | (1 << 4), 1))) return st;
    {
        fetd_sim::Timer t(s, 4);
        if ((st = sort_all(s, s->stream))) return st;
    }
    double ms[FETD_N_STAGES];
    int64_t n[FETD_N_STAGES];
    if ((st = fetd_stage_times(s, ms, n))) return st;
    const double t_sort = ms[4];
    if ((st = timed_particle_steps(s, pusher, trial_steps, tp))) return st;
    int best = saved;
    double best_cost = std::numeric_limits<double>::max();
    int ci = 0;
    for (int K : {5, 10, 20, 40, 80, 160}) {
        if (K <= trial_steps) {
            double sum = t_sort;
            for (int j = 0; j < K; ++j) sum += tp[j];
            const double cost = sum / K;
            if (out) out->resort_cost_ms[ci] = cost;
            if (cost < best_cost) {
                best_cost = cost;
                best = K;
            }
        }
        ++ci;
    }
    s->resort_every = best;
    s->steps_since_sort = trial_steps;  // the order has decayed: sort at the next step
    if ((st = fetd_profile_mask(s, was_mask, was_every))) return st;
    if (out) {
        out->resort_every = best;
        out->tile_particles = s->ppt * kBlock;
        out->scan_lanes = s->scan;
        out->defer_exits = s->fp32() ? s->defer : 1;
    }
    return FETD_OK;
}

fetd_status fetd_set_scan(fetd_sim *s, int32_t scan_lanes)
{
    if (!s) return FETD_E_ARG;
    return set_scan(s, scan_lanes);
}

fetd_status fetd_get_scan(fetd_sim *s, int32_t *scan_lanes)
{
    if (!s || !scan_lanes) return FETD_E_ARG;
    *scan_lanes = s->scan;
    return FETD_OK;
}

fetd_status fetd_set_defer_exits(fetd_sim *s, int32_t on)
{
    if (!s) return FETD_E_ARG;
    return set_defer(s, on);
}

fetd_status fetd_get_defer_exits(fetd_sim *s, int32_t *on)
{
    if (!s || !on) return FETD_E_ARG;
    *on = s->fp32() ? s->defer : 1;  // FP64 always defers
    return FETD_OK;
}

fetd_status fetd_set_tile(fetd_sim *s, int32_t tile_particles)
{
    if (!s) return FETD_E_ARG;
    if (tile_particles % kBlock != 0 || !valid_ppt(tile_particles / kBlock))
        return s->fail(FETD_E_ARG, "tile_particles must be a multiple of 256 from 512 to 2048");
    DeviceGuard g(s->device);
    return set_ppt(s, tile_particles / kBlock);
}

fetd_status fetd_get_tile(fetd_sim *s, int32_t *tile_particles)
{
    if (!s || !tile_particles) return FETD_E_ARG;
    *tile_particles = s->ppt * kBlock;
    return FETD_OK;
}

fetd_status fetd_copy_ceiling(int32_t device, int64_t bytes, int32_t reps, double *gbs)
{
    if (!gbs || bytes < (int64_t(1) << 20) || reps < 1) {
        g_last_error = "invalid copy-ceiling arguments";
        return FETD_E_ARG;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        g_last_error = "no such HIP device";
        return FETD_E_HIP;
    }
    DeviceGuard g(device);
    const int64_t n16 = bytes / 16;
    void *a = nullptr, *b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&a, size_t(n16) * 16);
    if (e == hipSuccess) e = hipMalloc(&b, size_t(n16) * 16);
    if (e == hipSuccess) e = hipMemset(a, 0x3c, size_t(n16) * 16);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    double best = 0.0;
    // the best of a few grid sizes, each timed `reps` times after one untimed launch
    for (int blocks : {512, 1024, 2048, 4096}) {
        for (int r = 0; r <= reps && e == hipSuccess; ++r) {
            e = hipEventRecord(e0, nullptr);
            if (e == hipSuccess) e = launch_copy(nullptr, a, b, n16, blocks);
            if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && r > 0 && ms > 0.f)
                best = std::max(best, 2.0 * double(n16) * 16.0 / (double(ms) * 1e-3) / 1e9);
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (e != hipSuccess) {
        g_last_error = std::string("copy ceiling: ") + hipGetErrorString(e);
        return FETD_E_HIP;
    }
    *gbs = best;
    return FETD_OK;
}

fetd_status fetd_info_get(fetd_sim *s, fetd_info *out)
{
    if (!s || !out) return FETD_E_ARG;
    out->n_nodes = s->nn;
    out->n_tris = s->nf;
    out->n_edges = s->ne;
    out->n_free_edges = s->n_free_e;
    out->n_free_nodes = s->n_free_n;
    out->spai_nnz = int64_t(s->mt.col.size());
    out->spai_frobenius = s->spai_fro;
    out->n_species = int32_t(s->species.size());
    out->device_bytes = s->device_bytes;
    return FETD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------
// Batched stepping.
// ---------------------------------------------------------------------
struct fetd_batch {
    std::vector<fetd_sim *> sims;
    hipStream_t member_stream = nullptr;  // the members' stream
    hipStream_t stream = nullptr;         // the batch's own stream (capturable)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    int device = 0;
    bool fp32 = false;
    bool det = false;
    bool use_graph = false;
    int nrun = 0, nseg = 0;
    uint32_t tri_blocks = 0, edge_blocks = 0, tiles = 0;
    FieldDesc *d_fields = nullptr;
    std::vector<FieldDesc> pml_fields;        // runs with a PML (their auxiliary launches)
    uint32_t *d_tri_prefix = nullptr, *d_edge_prefix = nullptr, *d_seg_prefix = nullptr;
    SegDesc *d_segs[2] = {nullptr, nullptr};  // [parity of sorts since creation]
    uint32_t *d_queue = nullptr;              // tile queue of the particle launch: [next, done]
    std::vector<int> pbuf0;                   // particle buffer of each run at creation
    std::vector<uint64_t> gen0;               // desc_gen of each run at the last build
    int parity = 0;
    int steps_since_sort = 0;
    int resort_every = 20;
    hipGraphExec_t graph = nullptr;
    int graph_pusher = -1;
    int graph_phase = -1;  // steps since the last sort (at most K) where the captured cycle starts
    int graph_parity = -1; // sort parity where it starts (its sorts read and write fixed buffers)
    unsigned warm = 0;  // pushers that have run an eager sorting step (all their kernels loaded)
    int64_t graph_captures = 0, graph_replays = 0, eager_steps = 0;
    std::string err;
};

namespace {

fetd_status batch_fail(fetd_batch *b, fetd_status st, const std::string &msg)
{
    b->err = msg;
    g_last_error = msg;
    return st;
}

template <typename T>
bool batch_upload(fetd_batch *b, T **dst, const std::vector<T> &v)
{
    void *p = nullptr;
    if (hipMalloc(&p, sizeof(T) * std::max<size_t>(1, v.size())) != hipSuccess) return false;
    *dst = static_cast<T *>(p);
    if (v.empty()) return true;
    return hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, b->stream) ==
               hipSuccess &&
           hipStreamSynchronize(b->stream) == hipSuccess;
}

SegDesc seg_desc(fetd_sim *s, const Species &sp, int pbuf)
{
    SegDesc d{};
    d.m = mesh_view(s);
    d.a = step_args(s, sp, pbuf);
    return d;
}

fetd_status batch_build(fetd_batch *b)
{
    std::vector<FieldDesc> fd;
    std::vector<uint32_t> tp(1, 0), ep(1, 0), sp(1, 0);
    std::vector<SegDesc> seg[2];
    // (tiles, run, species) of every non-empty segment, largest first, so
    // the tile queue hands out the longest runs before the short ones
    struct SegRef {
        int64_t tiles;
        int run, species;
    };
    std::vector<SegRef> refs;
    b->pml_fields.clear();
    for (size_t r = 0; r < b->sims.size(); ++r) {
        fetd_sim *s = b->sims[r];
        fd.push_back(field_desc(s));
        if (fd.back().pml_n > 0) b->pml_fields.push_back(fd.back());
        tp.push_back(tp.back() + uint32_t((s->nf + 255) / 256));
        ep.push_back(ep.back() + uint32_t((s->ne + 255) / 256));
        for (size_t k = 0; k < s->species.size(); ++k)
            if (s->species[k].n > 0)
                refs.push_back({tiles_of(s->species[k].n, s->ppt), int(r), int(k)});
    }
    std::stable_sort(refs.begin(), refs.end(),
                     [](const SegRef &x, const SegRef &y) { return x.tiles > y.tiles; });
    for (const SegRef &x : refs) {
        fetd_sim *s = b->sims[x.run];
        for (int par = 0; par < 2; ++par)
            seg[par].push_back(seg_desc(s, s->species[x.species], s->pbuf ^ par));
        sp.push_back(sp.back() + uint32_t(x.tiles));
    }
    b->nrun = int(b->sims.size());
    b->nseg = int(seg[0].size());
    b->tri_blocks = tp.back();
    b->edge_blocks = ep.back();
    b->tiles = sp.back();
    b->pbuf0.clear();
    b->gen0.clear();
    for (fetd_sim *s : b->sims) {
        b->pbuf0.push_back(s->pbuf);
        b->gen0.push_back(s->desc_gen);
    }
    b->parity = 0;
    const std::vector<uint32_t> queue0 = {0u, 0u};
    if (!batch_upload(b, &b->d_fields, fd) || !batch_upload(b, &b->d_tri_prefix, tp) ||
        !batch_upload(b, &b->d_edge_prefix, ep) || !batch_upload(b, &b->d_seg_prefix, sp) ||
        !batch_upload(b, &b->d_segs[0], seg[0]) || !batch_upload(b, &b->d_segs[1], seg[1]) ||
        !batch_upload(b, &b->d_queue, queue0))
        return batch_fail(b, FETD_E_OOM, "batch descriptors");
    return FETD_OK;
}

void batch_release(fetd_batch *b)
{
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    for (void *p : {(void *)b->d_fields, (void *)b->d_tri_prefix, (void *)b->d_edge_prefix,
                    (void *)b->d_seg_prefix, (void *)b->d_segs[0], (void *)b->d_segs[1],
                    (void *)b->d_queue})
        if (p) (void)hipFree(p);
    b->d_fields = nullptr;
    b->d_tri_prefix = b->d_edge_prefix = b->d_seg_prefix = nullptr;
    b->d_segs[0] = b->d_segs[1] = nullptr;
    b->d_queue = nullptr;
}

// Enqueue n batched steps (re-sorting when due) on the batch stream.
fetd_status batch_enqueue(fetd_batch *b, int n, int pusher)
{
    for (int it = 0; it < n; ++it) {
        bool sorted = false;
        if (b->steps_since_sort >= b->resort_every) {
            for (fetd_sim *s : b->sims)
                if (fetd_status st = sort_all(s, b->stream)) return batch_fail(b, st, s->err);
            b->parity ^= 1;
            b->steps_since_sort = 0;
            sorted = true;
        }
        hipError_t e = launch_faraday_batched(b->stream, b->d_fields, b->d_tri_prefix, b->nrun,
                                              b->tri_blocks);
        if (e == hipSuccess)
            e = launch_particles_batched(b->stream, b->d_segs[b->parity], b->d_seg_prefix, b->nseg,
                                         b->tiles, b->d_queue, pusher, b->fp32, b->det);
        if (e == hipSuccess)
            e = launch_ampere_batched(b->stream, b->d_fields, b->d_edge_prefix, b->nrun,
                                      b->edge_blocks);
        for (const FieldDesc &pf : b->pml_fields)
            if (e == hipSuccess) e = launch_pml_aux(b->stream, pf);
        if (e == hipSuccess)
            e = launch_spmv_batched(b->stream, b->d_fields, b->d_edge_prefix, b->nrun,
                                    b->edge_blocks);
        if (e != hipSuccess) return batch_fail(b, FETD_E_HIP, hipGetErrorString(e));
        ++b->steps_since_sort;
        for (fetd_sim *s : b->sims) {
            ++s->step;
            s->steps_since_sort = b->steps_since_sort;
        }
        // a sorting step launches every kernel of a cycle; outside a
        // capture that loads them, so later calls may capture at once
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (sorted && hipStreamIsCapturing(b->stream, &cs) == hipSuccess &&
            cs == hipStreamCaptureStatusNone)
            b->warm |= 1u << pusher;
    }
    return FETD_OK;
}

// Steps of a batch call in graph mode.  A cycle of 2K steps (K the re-sort
// interval) from any phase (steps since the last sort) holds two sorts and
// returns the particle buffers, the sort parity and the phase to where they
// were, so it is captured once per pusher and phase and replayed.  Before a
// pusher's first capture the batch runs eagerly up to and including a
// sorting step (every kernel of a cycle is then loaded, which a capture
// forbids doing).  A call that replays the existing graph at the current
// phase does so at once; otherwise a call long enough first runs eagerly up
// to the next sort (so graphs start right before a sort) and a shorter one
// captures at the current phase, so a batch stepped in calls of 2K steps
// replays from its third call at the latest.  The rest runs eagerly.
fetd_status batch_graph_steps(fetd_batch *b, int left, int pusher)
{
    const int K = b->resort_every;
    const int cycle = 2 * K;
    if (left >= cycle && !((b->warm >> pusher) & 1u)) {
        const int n = std::min(left, std::max(1, K - b->steps_since_sort + 1));
        if (fetd_status st = batch_enqueue(b, n, pusher)) return st;
        b->eager_steps += n;
        left -= n;
    }
    if (left >= cycle && ((b->warm >> pusher) & 1u)) {
        int phase = std::min(b->steps_since_sort, K);
        const bool same = b->graph && b->graph_pusher == pusher && b->graph_phase == phase &&
                          b->graph_parity == b->parity;
        const int lead = K - phase;
        if (!same && lead > 0 && left >= lead + cycle) {
            if (fetd_status st = batch_enqueue(b, lead, pusher)) return st;
            b->eager_steps += lead;
            left -= lead;
            phase = K;
        }
        if (b->graph && (b->graph_pusher != pusher || b->graph_phase != phase ||
                         b->graph_parity != b->parity)) {
            (void)hipGraphExecDestroy(b->graph);
            b->graph = nullptr;
        }
        if (!b->graph) {
            // capture with the host counters advanced as during replay
            const int save_parity = b->parity, save_since = b->steps_since_sort;
            std::vector<int64_t> save_step, save_since_sim;
            std::vector<int> save_pbuf;
            for (fetd_sim *s : b->sims) {
                save_step.push_back(s->step);
                save_since_sim.push_back(s->steps_since_sort);
                save_pbuf.push_back(s->pbuf);
            }
            hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return batch_fail(b, FETD_E_HIP, hipGetErrorString(e));
            fetd_status st = batch_enqueue(b, cycle, pusher);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(b->stream, &graph);
            b->parity = save_parity;
            b->steps_since_sort = save_since;
            for (size_t r = 0; r < b->sims.size(); ++r) {
                b->sims[r]->step = save_step[r];
                b->sims[r]->steps_since_sort = save_since_sim[r];
                b->sims[r]->pbuf = save_pbuf[r];
            }
            if (st) {
                if (graph) (void)hipGraphDestroy(graph);
                return st;
            }
            if (e != hipSuccess) return batch_fail(b, FETD_E_HIP, hipGetErrorString(e));
            e = hipGraphInstantiate(&b->graph, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return batch_fail(b, FETD_E_HIP, hipGetErrorString(e));
            b->graph_pusher = pusher;
            b->graph_phase = phase;
            b->graph_parity = b->parity;
            ++b->graph_captures;
        }
        while (left >= cycle) {
            hipError_t e = hipGraphLaunch(b->graph, b->stream);
            if (e != hipSuccess) return batch_fail(b, FETD_E_HIP, hipGetErrorString(e));
            for (fetd_sim *s : b->sims) {
                s->step += cycle;
                s->steps_since_sort = phase;
            }
            b->steps_since_sort = phase;
            ++b->graph_replays;
            left -= cycle;
        }
    }
    if (fetd_status st = batch_enqueue(b, left, pusher)) return st;
    b->eager_steps += left;
    return FETD_OK;
}

}  // namespace

extern "C" {

fetd_status fetd_batch_create(fetd_sim *const *sims, int32_t n, int32_t use_graph,
                              fetd_batch **out)
{
    if (!out || !sims || n <= 0) {
        g_last_error = "invalid batch arguments";
        return FETD_E_ARG;
    }
    *out = nullptr;
    for (int32_t i = 0; i < n; ++i)
        if (!sims[i]) {
            g_last_error = "invalid batch arguments";
            return FETD_E_ARG;
        }
    {
        std::vector<fetd_sim *> seen(sims, sims + n);
        std::sort(seen.begin(), seen.end());
        if (std::adjacent_find(seen.begin(), seen.end()) != seen.end()) {
            g_last_error = "a simulation appears twice in the batch";
            return FETD_E_ARG;
        }
    }
    fetd_batch *b = new (std::nothrow) fetd_batch();
    if (!b) return FETD_E_OOM;
    b->sims.assign(sims, sims + n);
    b->member_stream = sims[0]->stream;
    b->device = sims[0]->device;
    b->fp32 = sims[0]->fp32();
    b->det = sims[0]->deterministic;
    b->use_graph = use_graph != 0;
    b->resort_every = sims[0]->resort_every;
    for (fetd_sim *s : b->sims) {
        if (s->stream != b->member_stream || s->device != b->device || s->fp32() != b->fp32 ||
            s->deterministic != b->det) {
            delete b;
            g_last_error = "batch members must share device, stream, precision and determinism";
            return FETD_E_ARG;
        }
    }
    DeviceGuard g(b->device);
    // The batch works on a stream of its own (a non-blocking one, so a HIP
    // graph can be captured on it even when the members use the legacy
    // default stream) and hands over to and from the members' stream with
    // events at every call.
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess) {
        fetd_batch_destroy(b);
        g_last_error = "batch stream";
        return FETD_E_HIP;
    }
    for (fetd_sim *s : b->sims) {
        if (!s->have_baseline)
            if (fetd_status st = take_baseline(s)) {
                g_last_error = s->err;
                fetd_batch_destroy(b);
                return st;
            }
    }
    if (hipStreamSynchronize(b->member_stream) != hipSuccess) {
        fetd_batch_destroy(b);
        g_last_error = "member stream";
        return FETD_E_HIP;
    }
    b->steps_since_sort = 0;
    for (fetd_sim *s : b->sims) b->steps_since_sort = std::max<int>(b->steps_since_sort, int(s->steps_since_sort));
    if (fetd_status st = batch_build(b)) {
        fetd_batch_destroy(b);
        return st;
    }
    *out = b;
    return FETD_OK;
}

fetd_status fetd_batch_step(fetd_batch *b, int32_t n_steps, int32_t pusher)
{
    if (!b || n_steps < 0 || pusher < 0 || pusher > 3) return FETD_E_ARG;
    DeviceGuard g(b->device);
    // the members may have been sorted, reloaded or given new applied
    // fields or layers individually: rebuild the descriptors
    bool stale = false;
    for (size_t r = 0; r < b->sims.size(); ++r)
        if ((b->sims[r]->pbuf ^ b->parity) != b->pbuf0[r] || b->sims[r]->desc_gen != b->gen0[r])
            stale = true;
    if (stale) {
        if (hipError_t e = hipStreamSynchronize(b->stream))
            return batch_fail(b, FETD_E_HIP, hipGetErrorString(e));
        batch_release(b);
        if (fetd_status st = batch_build(b)) return st;
    }
    // members' work first, the batch's after it, the members' next work after that
    hipError_t e = hipEventRecord(b->ev_in, b->member_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_in, 0);
    if (e != hipSuccess) return batch_fail(b, FETD_E_HIP, hipGetErrorString(e));
    fetd_status st;
    if (b->use_graph) {
        st = batch_graph_steps(b, n_steps, pusher);
    } else {
        st = batch_enqueue(b, n_steps, pusher);
        if (!st) b->eager_steps += n_steps;
    }
    e = hipEventRecord(b->ev_out, b->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->member_stream, b->ev_out, 0);
    if (!st && e != hipSuccess) return batch_fail(b, FETD_E_HIP, hipGetErrorString(e));
    return st;
}

fetd_status fetd_batch_stats(fetd_batch *b, int64_t *graph_captures, int64_t *graph_replays,
                             int64_t *eager_steps)
{
    if (!b) return FETD_E_ARG;
    if (graph_captures) *graph_captures = b->graph_captures;
    if (graph_replays) *graph_replays = b->graph_replays;
    if (eager_steps) *eager_steps = b->eager_steps;
    return FETD_OK;
}

void fetd_batch_destroy(fetd_batch *b)
{
    if (!b) return;
    DeviceGuard g(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    batch_release(b);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // extern "C"

// ---------------------------------------------------------------------
// Batched stepping without allocation.
//
// fetd_batch_step_noalloc steps a list of simulations together with the
// batched kernels, like fetd_batch_step, but needs no batch object: the
// tables those kernels read (per-run field descriptors, per-segment particle
// descriptors for both sort parities, block and tile prefix tables, the tile
// queue) go to `scratch`, a fixed device array of the library, instead of
// device memory allocated per batch.  Every call on a device shares that
// device's copy and rewrites it, so calls that overlap on one device race.
// ---------------------------------------------------------------------
namespace {

constexpr int kNoAllocRuns = 256;
constexpr int kNoAllocSegs = 512;
constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
constexpr size_t kOffFields = 0;
constexpr size_t kOffSegs0 = align256(kOffFields + sizeof(FieldDesc) * kNoAllocRuns);
constexpr size_t kOffSegs1 = align256(kOffSegs0 + sizeof(SegDesc) * kNoAllocSegs);
constexpr size_t kOffTriPrefix = align256(kOffSegs1 + sizeof(SegDesc) * kNoAllocSegs);
constexpr size_t kOffEdgePrefix = align256(kOffTriPrefix + 4 * size_t(kNoAllocRuns + 1));
constexpr size_t kOffSegPrefix = align256(kOffEdgePrefix + 4 * size_t(kNoAllocRuns + 1));
constexpr size_t kOffQueue = align256(kOffSegPrefix + 4 * size_t(kNoAllocSegs + 1));
constexpr size_t kScratchBytes = align256(kOffQueue + 2 * sizeof(uint32_t));
static_assert(kScratchBytes <= 393216, "scratch stays at 384 KiB");

}  // namespace

// The library's fixed device array for fetd_batch_step_noalloc (one copy
// per device, held until the process ends).  Host code must not pass this
// name to a kernel or a copy: it uses the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_noalloc_mu;          // host staging tables and the address cache
void *g_scratch_dev[64] = {};     // device address of `scratch` per device ordinal

struct NoAllocStaging {
    FieldDesc fields[kNoAllocRuns];
    SegDesc segs[2][kNoAllocSegs];
    uint32_t tri_prefix[kNoAllocRuns + 1];
    uint32_t edge_prefix[kNoAllocRuns + 1];
    uint32_t seg_prefix[kNoAllocSegs + 1];
    int seg_run[kNoAllocSegs], seg_species[kNoAllocSegs];
    int64_t seg_tiles[kNoAllocSegs];
};
NoAllocStaging g_staging;

// Device address of `scratch` on `device` (the current device), looked up
// once per device.
hipError_t scratch_address(int device, char **out)
{
    if (device < 0 || device >= 64) return hipErrorInvalidDevice;
    if (!g_scratch_dev[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_dev[device] = p;
    }
    *out = static_cast<char *>(g_scratch_dev[device]);
    return hipSuccess;
}

}  // namespace

extern "C" fetd_status fetd_batch_step_noalloc(fetd_sim *const *sims, int32_t n, int32_t n_steps,
                                               int32_t pusher)
{
    if (!sims || n <= 0 || n_steps < 0 || pusher < 0 || pusher > 3) {
        g_last_error = "invalid batch arguments";
        return FETD_E_ARG;
    }
    for (int32_t i = 0; i < n; ++i)
        if (!sims[i]) {
            g_last_error = "invalid batch arguments";
            return FETD_E_ARG;
        }
    fetd_sim *s0 = sims[0];
    int nseg = 0;
    for (int32_t i = 0; i < n; ++i) {
        fetd_sim *s = sims[i];
        if (s->stream != s0->stream || s->device != s0->device || s->fp32() != s0->fp32() ||
            s->deterministic != s0->deterministic) {
            g_last_error = "batch members must share device, stream, precision and determinism";
            return FETD_E_ARG;
        }
        for (const Species &sp : s->species) nseg += sp.n > 0 ? 1 : 0;
    }
    if (n > kNoAllocRuns || nseg > kNoAllocSegs) {
        g_last_error = "fetd_batch_step_noalloc: more than 256 runs or 512 species segments";
        return FETD_E_ARG;
    }
    if (n_steps == 0) return FETD_OK;
    DeviceGuard g(s0->device);
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    char *base = nullptr;
    if (hipError_t e = scratch_address(s0->device, &base)) {
        g_last_error = std::string("scratch address: ") + hipGetErrorString(e);
        return FETD_E_HIP;
    }
    // descriptor tables (as fetd_batch_create builds them), segments largest first
    NoAllocStaging &h = g_staging;
    h.tri_prefix[0] = h.edge_prefix[0] = h.seg_prefix[0] = 0;
    int k = 0;
    for (int32_t r = 0; r < n; ++r) {
        fetd_sim *s = sims[r];
        h.fields[r] = field_desc(s);
        h.tri_prefix[r + 1] = h.tri_prefix[r] + uint32_t((s->nf + 255) / 256);
        h.edge_prefix[r + 1] = h.edge_prefix[r] + uint32_t((s->ne + 255) / 256);
        for (size_t q = 0; q < s->species.size(); ++q)
            if (s->species[q].n > 0) {
                h.seg_run[k] = r;
                h.seg_species[k] = int(q);
                h.seg_tiles[k] = tiles_of(s->species[q].n, s->ppt);
                ++k;
            }
    }
    // stable selection order by tile count, largest first (insertion sort:
    // no allocation)
    int order[kNoAllocSegs];
    for (int i = 0; i < nseg; ++i) {
        int j = i;
        while (j > 0 && h.seg_tiles[order[j - 1]] < h.seg_tiles[i]) {
            order[j] = order[j - 1];
            --j;
        }
        order[j] = i;
    }
    for (int i = 0; i < nseg; ++i) {
        const int q = order[i];
        fetd_sim *s = sims[h.seg_run[q]];
        const Species &sp = s->species[h.seg_species[q]];
        for (int par = 0; par < 2; ++par) h.segs[par][i] = seg_desc(s, sp, s->pbuf ^ par);
        h.seg_prefix[i + 1] = h.seg_prefix[i] + uint32_t(h.seg_tiles[q]);
    }
    const hipStream_t stream = s0->stream;
    FieldDesc *d_fields = reinterpret_cast<FieldDesc *>(base + kOffFields);
    SegDesc *d_segs[2] = {reinterpret_cast<SegDesc *>(base + kOffSegs0),
                          reinterpret_cast<SegDesc *>(base + kOffSegs1)};
    uint32_t *d_tp = reinterpret_cast<uint32_t *>(base + kOffTriPrefix);
    uint32_t *d_ep = reinterpret_cast<uint32_t *>(base + kOffEdgePrefix);
    uint32_t *d_sp = reinterpret_cast<uint32_t *>(base + kOffSegPrefix);
    uint32_t *d_queue = reinterpret_cast<uint32_t *>(base + kOffQueue);
    // the copies read the host staging tables: wait for them before the
    // staging can be rebuilt by a later call
    hipError_t e = hipMemcpyAsync(d_fields, h.fields, sizeof(FieldDesc) * n,
                                  hipMemcpyHostToDevice, stream);
    for (int par = 0; par < 2 && e == hipSuccess; ++par)
        e = hipMemcpyAsync(d_segs[par], h.segs[par], sizeof(SegDesc) * size_t(nseg),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_tp, h.tri_prefix, 4 * size_t(n + 1), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_ep, h.edge_prefix, 4 * size_t(n + 1), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_sp, h.seg_prefix, 4 * size_t(nseg + 1), hipMemcpyHostToDevice,
                           stream);
    // the tile queue starts at zero (a fill kernel, no memset node)
    if (e == hipSuccess) e = launch_fill_u32(stream, d_queue, 0u, 2);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        g_last_error = std::string("fetd_batch_step_noalloc upload: ") + hipGetErrorString(e);
        return FETD_E_HIP;
    }
    // steps: the re-sort interval of the first simulation, counted from the
    // members' largest steps-since-sort (as a batch does)
    const int K = s0->resort_every;
    int since = 0;
    for (int32_t i = 0; i < n; ++i) since = std::max<int>(since, int(sims[i]->steps_since_sort));
    int parity = 0;
    const uint32_t tri_blocks = h.tri_prefix[n], edge_blocks = h.edge_prefix[n];
    const uint32_t tiles = h.seg_prefix[nseg];
    for (int it = 0; it < n_steps; ++it) {
        if (since >= K) {
            for (int32_t i = 0; i < n; ++i)
                if (fetd_status st = sort_all(sims[i], stream)) {
                    g_last_error = sims[i]->err;
                    return st;
                }
            parity ^= 1;
            since = 0;
        }
        e = launch_faraday_batched(stream, d_fields, d_tp, n, tri_blocks);
        if (e == hipSuccess)
            e = launch_particles_batched(stream, d_segs[parity], d_sp, nseg, tiles, d_queue, pusher,
                                         s0->fp32(), s0->deterministic);
        if (e == hipSuccess) e = launch_ampere_batched(stream, d_fields, d_ep, n, edge_blocks);
        for (int32_t r = 0; r < n && e == hipSuccess; ++r)
            if (h.fields[r].pml_n > 0) e = launch_pml_aux(stream, h.fields[r]);
        if (e == hipSuccess) e = launch_spmv_batched(stream, d_fields, d_ep, n, edge_blocks);
        if (e != hipSuccess) {
            g_last_error = std::string("fetd_batch_step_noalloc: ") + hipGetErrorString(e);
            return FETD_E_HIP;
        }
        ++since;
        for (int32_t i = 0; i < n; ++i) {
            ++sims[i]->step;
            sims[i]->steps_since_sort = since;
        }
    }
    return FETD_OK;
}
