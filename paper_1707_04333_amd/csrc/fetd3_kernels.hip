// HIP kernels (gfx950) of the tetrahedral FETD-PIC path, FP64:
//   k3_faraday    b^{n+1/2} = b^{n-1/2} - dt C e^n and the face average
//                 (b^{n+1/2} + b^{n-1/2})/2 (Sec. II.A, eq. semi.dis.curl.1)
//   k3_record     per-tetrahedron gather record: E = sum l_n V_n from the
//                 Whitney 1-forms of the six edges, B = sum l_n U_n from the
//                 Whitney 2-forms of the four faces (Sec. II.B)
//   k3_particles  gather, push (Sec. II.C, four pushers), move with face
//                 crossings and the charge-conserving W1 deposit of every
//                 piece on its six edges (Sec. II.D, eq. I.assign)
//   k3_hnu, k3_ampere, k3_spmv   h = [*mu^-1] b, d += dt (C^T h - i),
//                 e = M~ d (Sec. II.A, eq. semi.dis.curl.2 in the d form)
//   k3_sort_*     counting sort of the particles by tetrahedron
#include "fetd3_internal.h"
#include "stage_events.h"

namespace fetd3 {
namespace {

__device__ __forceinline__ void atomic_add_f64(double *p, double v) { unsafeAtomicAdd(p, v); }

// Blocks are dispatched round-robin over the 8 XCDs, each with its own L2:
// give each XCD a contiguous run of particle blocks, so that the
// tetrahedron tables a run of sorted particles shares stay in one L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb)
{
    const int64_t x = b & 7, j = b >> 3;
    const int64_t per = nb >> 3, rem = nb & 7;
    return x < rem ? x * (per + 1) + j : rem * (per + 1) + (x - rem) * per + j;
}

inline unsigned grid_for(int64_t n, int b) { return unsigned((n + b - 1) / b); }

// value of a[i] for a runtime i in 0..3 without dynamic indexing
__device__ __forceinline__ double pick4(const double (&a)[4], int i)
{
    return i == 0 ? a[0] : i == 1 ? a[1] : i == 2 ? a[2] : a[3];
}

__device__ __forceinline__ void put4(double (&a)[4], int i, double v)
{
    a[0] = i == 0 ? v : a[0];
    a[1] = i == 1 ? v : a[1];
    a[2] = i == 2 ? v : a[2];
    a[3] = i == 3 ? v : a[3];
}

// The four barycentrics from the stored triple of slot r.
__device__ __forceinline__ void unpack_lambda(int r, double s0, double s1, double s2,
                                              double (&L)[4])
{
    const double lr = ((1.0 - s0) - s1) - s2;
    L[0] = L[1] = L[2] = L[3] = 0.0;
    put4(L, r, lr);
    put4(L, (r + 1) & 3, s0);
    put4(L, (r + 2) & 3, s1);
    put4(L, (r + 3) & 3, s2);
}

__global__ __launch_bounds__(256) void k3_faraday(int nf, const int4 *__restrict__ face_edge,
                                                  const double *__restrict__ e,
                                                  double *__restrict__ b,
                                                  double *__restrict__ bavg, double dt)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    const int4 fe = face_edge[f];
    // C row: +1 on edges (i,j) and (j,l), -1 on (i,l) (bits of fe.w)
    const double c0 = (fe.w & 1) ? -e[fe.x] : e[fe.x];
    const double c1 = (fe.w & 2) ? -e[fe.y] : e[fe.y];
    const double c2 = (fe.w & 4) ? -e[fe.z] : e[fe.z];
    const double bo = b[f];
    const double bn = bo - dt * ((c0 + c1) + c2);
    b[f] = bn;
    bavg[f] = 0.5 * (bn + bo);
}

template <typename R>
__global__ __launch_bounds__(256) void k3_record(int nt, Mesh3 m, const double *__restrict__ e,
                                                 const double *__restrict__ e_ext,
                                                 const double *__restrict__ bavg,
                                                 R *__restrict__ rec)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const int32_t *te = m.tet_edge + 8 * size_t(t);
    const int bits = te[6];
    double g[12];
    for (int i = 0; i < 12; ++i) g[i] = m.grad[12 * size_t(t) + i];
    double V[12], U[12];
    for (int i = 0; i < 12; ++i) V[i] = U[i] = 0.0;
    // E = sum_k s_k e_k (l_a grad l_b - l_b grad l_a) = sum_n l_n V_n
    constexpr int ea[6] = {0, 0, 0, 1, 1, 2}, eb[6] = {1, 2, 3, 2, 3, 3};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        double dof = e[te[k]];
        if (e_ext) dof = dof + e_ext[te[k]];
        const double tk = ((bits >> k) & 1) ? -dof : dof;
        const int a = ea[k], b = eb[k];
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            V[3 * a + x] += tk * g[3 * b + x];
            V[3 * b + x] -= tk * g[3 * a + x];
        }
    }
    // B = sum_k p_k b_k 2 (l_p X_qr + l_q X_rp + l_r X_pq) = sum_n l_n U_n
    const int4 tf = m.tet_face[t];
    const int fid[4] = {tf.x, tf.y, tf.z, tf.w};
    constexpr int fp[4] = {1, 0, 0, 0}, fq[4] = {2, 2, 1, 1}, fr[4] = {3, 3, 3, 2};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double bk = bavg[fid[k]];
        const double beta = 2.0 * (((bits >> (8 + k)) & 1) ? -bk : bk);
        const int p = fp[k], q = fq[k], r = fr[k];
        const double *gp = g + 3 * p, *gq = g + 3 * q, *gr = g + 3 * r;
        const double xqr[3] = {gq[1] * gr[2] - gq[2] * gr[1], gq[2] * gr[0] - gq[0] * gr[2],
                               gq[0] * gr[1] - gq[1] * gr[0]};
        const double xrp[3] = {gr[1] * gp[2] - gr[2] * gp[1], gr[2] * gp[0] - gr[0] * gp[2],
                               gr[0] * gp[1] - gr[1] * gp[0]};
        const double xpq[3] = {gp[1] * gq[2] - gp[2] * gq[1], gp[2] * gq[0] - gp[0] * gq[2],
                               gp[0] * gq[1] - gp[1] * gq[0]};
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            U[3 * p + x] += beta * xqr[x];
            U[3 * q + x] += beta * xrp[x];
            U[3 * r + x] += beta * xpq[x];
        }
    }
    R *o = rec + size_t(kRec) * t;
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        o[i] = R(V[i]);
        o[12 + i] = R(U[i]);
    }
}

// ---------------------------------------------------------------------
// Pushers (Sec. II.C) for general 3-vectors; eps = alpha E, beta = alpha B.
// ---------------------------------------------------------------------
template <typename R>
struct V3 {
    R x, y, z;
};
template <typename R>
__device__ __forceinline__ V3<R> operator+(V3<R> a, V3<R> b)
{
    return {a.x + b.x, a.y + b.y, a.z + b.z};
}
template <typename R>
__device__ __forceinline__ V3<R> operator*(R s, V3<R> a)
{
    return {s * a.x, s * a.y, s * a.z};
}
template <typename R>
__device__ __forceinline__ R dot(V3<R> a, V3<R> b)
{
    return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename R>
__device__ __forceinline__ V3<R> cross(V3<R> a, V3<R> b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// gamma of a momentum: sqrt(1 + |u|^2 / c^2)
template <typename R>
__device__ __forceinline__ R gam(V3<R> u, R inv_c2)
{
    return sqrt(R(1) + dot(u, u) * inv_c2);
}

// One momentum update in the precision R (FP64, or FP32 in the mixed mode).
template <int P, typename R>
__device__ __forceinline__ V3<R> push3(V3<R> u, V3<R> eps, V3<R> beta, R c, R inv_c2)
{
    const R one = R(1);
    if constexpr (P == 2) {
        // Vay: u' = u + 2 eps + v x beta; gamma+ from the implicit midpoint
        // equation; u = s [u' + (u'.t) t + u' x t], t = beta/gamma+.
        const R g = gam(u, inv_c2);
        const V3<R> v = (one / g) * u;
        const V3<R> upr = (u + eps + cross(v, beta)) + eps;
        const R gp = gam(upr, inv_c2);
        const R bb = dot(beta, beta);
        const R sig = gp * gp - bb;
        const R us = dot(upr, beta) / c;
        const R gn = sqrt(R(0.5) * (sig + sqrt(sig * sig + R(4) * (bb + us * us))));
        const V3<R> t = (one / gn) * beta;
        const R sv = one / (one + dot(t, t));
        return sv * ((upr + dot(upr, t) * t) + cross(upr, t));
    } else {
        const V3<R> um = u + eps;
        R gbar;
        if constexpr (P == 3) {
            // Higuera-Cary: gamma of the midpoint momentum
            const R bb = dot(beta, beta);
            const R gm = gam(um, inv_c2);
            const R sig = gm * gm - bb;
            const R w = dot(beta, um) / c;
            gbar = sqrt(R(0.5) * (sig + sqrt(sig * sig + R(4) * (bb + w * w))));
        } else {
            gbar = gam(um, inv_c2);
        }
        V3<R> t;
        if constexpr (P == 1) {
            // Boris with the tangent correction of the rotation angle
            const R bm = sqrt(dot(beta, beta));
            t = bm > R(0) ? (tan(bm / gbar) / bm) * beta : V3<R>{R(0), R(0), R(0)};
        } else {
            t = (one / gbar) * beta;
        }
        const V3<R> s = (R(2) / (one + dot(t, t))) * t;
        const V3<R> up = um + cross(um, t);
        return (um + cross(up, s)) + eps;
    }
}

// Block-local FP64 current accumulation: kWin3 consecutive device edge ids
// in LDS around the block's home tetrahedron, and a small open-addressing
// table for the edges outside it (an edge shared with a tetrahedron far
// away in the tetrahedron order); only when the table's probes are taken
// does an add go straight to the global accumulator.
struct Window3 {
    double *acc;
    int *hkey;     // [kHash3], -1 = free
    double *hval;  // [kHash3]
    double *global;
    int base;

    __device__ __forceinline__ void add(int edge, double v) const
    {
        const unsigned j = unsigned(edge - base);
        if (j < unsigned(kWin3)) {
            __hip_atomic_fetch_add(acc + j, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            return;
        }
        const unsigned h = (unsigned(edge) * 2654435761u) >> (32 - kHashBits3);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const unsigned slot = (h + unsigned(q)) & unsigned(kHash3 - 1);
            int k = hkey[slot];
            if (k == -1) {
                k = atomicCAS(hkey + slot, -1, edge);
                if (k == -1) k = edge;
            }
            if (k == edge) {
                __hip_atomic_fetch_add(hval + slot, v, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                return;
            }
        }
        atomic_add_f64(global + edge, v);
    }
};

// Current of one piece inside tetrahedron t from Ls to Lf: i_e += sign
// (Q/dt) (l_a^s l_b^f - l_a^f l_b^s) on each local edge (a, b).
__device__ __forceinline__ void deposit_piece(const int32_t *__restrict__ te, int bits,
                                              const double (&Ls)[4], const double (&Lf)[4],
                                              double qdt, const Window3 &win)
{
    constexpr int ea[6] = {0, 0, 0, 1, 1, 2}, eb[6] = {1, 2, 3, 2, 3, 3};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int a = ea[k], b = eb[k];
        const double w = Ls[a] * Lf[b] - Lf[a] * Ls[b];
        const double sq = ((bits >> k) & 1) ? -qdt : qdt;
        win.add(te[k], sq * w);
    }
}

// Cross-lane move of a double by a DPP control; lanes whose source lies
// outside the row (or in a row disabled by RM) read 0.
template <int CTRL, int RM>
__device__ __forceinline__ double dpp_f64(double v)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, RM, 0xF, true);
    hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, RM, 0xF, true);
    return __hiloint2double(hi, lo);
}

template <int CTRL, int RM>
__device__ __forceinline__ void seg_step6(double (&c)[6], bool take)
{
    double o[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) o[k] = dpp_f64<CTRL, RM>(c[k]);
    if (take)
#pragma unroll
        for (int k = 0; k < 6; ++k) c[k] += o[k];
}

// Inclusive segmented sum over the wavefront: every lane ends with the sum
// over its run [seg_start, lane] (row shifts 1, 2, 4, 8 inside rows of 16
// lanes, then the row-15 and row-31 broadcasts across rows).
__device__ __forceinline__ void wave_segmented_sum6(double (&c)[6], int lane, int seg_start)
{
    const int in_row = lane & 15;
    seg_step6<0x111, 0xF>(c, in_row >= 1 && lane - 1 >= seg_start);
    seg_step6<0x112, 0xF>(c, in_row >= 2 && lane - 2 >= seg_start);
    seg_step6<0x114, 0xF>(c, in_row >= 4 && lane - 4 >= seg_start);
    seg_step6<0x118, 0xF>(c, in_row >= 8 && lane - 8 >= seg_start);
    seg_step6<0x142, 0xA>(c, (lane & 16) && (lane & ~15) - 1 >= seg_start);
    seg_step6<0x143, 0xC>(c, lane >= 32 && 31 >= seg_start);
}

// Exit test of one piece: dL_k = grad l_k . r for the four faces, the face
// with the smallest tau_k = max(l_k, 0)/(-dL_k) among dL_k < 0 (not the
// face just entered; ties to the smaller k), or ks = -1.
template <typename R>
__device__ __forceinline__ void exit_face(const R *__restrict__ G, R rx, R ry, R rz,
                                          const double (&L)[4], int entry, R (&dL)[4], int &ks,
                                          R &ts)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) dL[k] = G[3 * k] * rx + G[3 * k + 1] * ry + G[3 * k + 2] * rz;
    ks = -1;
    ts = R(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k == entry || !(dL[k] < R(0))) continue;
        const R lk = R(L[k]);
        const R tk = (lk > R(0) ? lk : R(0)) / (-dL[k]);
        if (ks < 0 || tk < ts) {
            ks = k;
            ts = tk;
        }
    }
}

// value of a[i] for a runtime i in 0..3 (precision R)
template <typename R>
__device__ __forceinline__ R pickR(const R (&a)[4], int i)
{
    return i == 0 ? a[0] : i == 1 ? a[1] : i == 2 ? a[2] : a[3];
}

// W1 weights l_a^s l_b^f - l_a^f l_b^s of the six local edges of a piece.
__device__ __forceinline__ void piece_weights(const double (&Ls)[4], const double (&Lf)[4],
                                              double (&w)[6])
{
    constexpr int ea[6] = {0, 0, 0, 1, 1, 2}, eb[6] = {1, 2, 3, 2, 3, 3};
#pragma unroll
    for (int k = 0; k < 6; ++k) w[k] = Ls[ea[k]] * Lf[eb[k]] - Lf[ea[k]] * Ls[eb[k]];
}

// Continue a particle that crossed a face: march and deposit piece by piece
// (pieces 2, 3, ... of the step).  Barycentrics are carried in FP64 so that
// every piece ends where the next one starts and they sum to 1 exactly;
// the march itself runs in the precision R.
template <typename R>
__device__ __forceinline__ void continue_move(const Mesh3 &m, const Step3 &a, const Window3 &win,
                                              const R *__restrict__ grad, int64_t p, int t, int r,
                                              int entry, double (&L)[4], R rx, R ry, R rz,
                                              unsigned long long &pieces,
                                              unsigned long long &lost_here)
{
    const int64_t n = a.stride;
    R *lam = static_cast<R *>(a.lam);
    bool fin = false;
    for (int it = 1; it < a.cap; ++it) {
        const int32_t *te = m.tet_edge + 8 * size_t(t);
        const int bits = te[6];
        R dL[4];
        int ks;
        R ts;
        exit_face(grad + 12 * size_t(t), rx, ry, rz, L, entry, dL, ks, ts);
        double Lf[4];
        ++pieces;
        if (ks < 0 || ts >= R(1)) {
            const int i1 = (r + 1) & 3, i2 = (r + 2) & 3, i3 = (r + 3) & 3;
            const R f1 = R(pick4(L, i1)) + pickR(dL, i1);
            const R f2 = R(pick4(L, i2)) + pickR(dL, i2);
            const R f3 = R(pick4(L, i3)) + pickR(dL, i3);
            unpack_lambda(r, double(f1), double(f2), double(f3), Lf);
            deposit_piece(te, bits, L, Lf, a.qdt, win);
            a.key[p] = uint32_t(t) | (uint32_t(r) << 30);
            lam[p] = f1;
            lam[n + p] = f2;
            lam[2 * n + p] = f3;
            fin = true;
            break;
        }
        const int kp = (ks + 1) & 3, kq = (ks + 2) & 3, kw = (ks + 3) & 3;
        const R lp = R(pick4(L, kp)) + ts * pickR(dL, kp);
        const R lq = R(pick4(L, kq)) + ts * pickR(dL, kq);
        const double lw = (1.0 - double(lp)) - double(lq);
        Lf[0] = Lf[1] = Lf[2] = Lf[3] = 0.0;
        put4(Lf, kp, double(lp));
        put4(Lf, kq, double(lq));
        put4(Lf, kw, lw);
        deposit_piece(te, bits, L, Lf, a.qdt, win);
        const int4 nb4 = m.tet_nbr[t];
        const int nb = ks == 0 ? nb4.x : ks == 1 ? nb4.y : ks == 2 ? nb4.z : nb4.w;
        if (nb < 0) {
            // wall: removed after depositing up to it
            a.key[p] = kLost;
            ++lost_here;
            fin = true;
            break;
        }
        const uint32_t mp = (m.tet_map[t] >> (8 * ks)) & 0xFFu;
        L[0] = L[1] = L[2] = L[3] = 0.0;
        put4(L, int(mp & 3), double(lp));
        put4(L, int((mp >> 2) & 3), double(lq));
        put4(L, int((mp >> 4) & 3), lw);
        r = int((mp >> 4) & 3);
        entry = int(mp >> 6);
        t = nb;
        const R sc = R(1) - ts;
        rx *= sc;
        ry *= sc;
        rz *= sc;
    }
    if (!fin) {
        atomicOr(a.counters + 2, 1ull);
        atomicMin(a.counters + 3, (unsigned long long)p);
    }
}

// One particle block: phase A (every lane: gather, push, first piece), a
// wavefront sum of the first-piece currents over runs of equal start
// tetrahedron (particles are sorted by tetrahedron), then phase B for the
// particles that crossed a face, depositing piece by piece.  R is the
// precision of the particle state, gather, push and march (FP64, or FP32 in
// the mixed mode); barycentrics in flight and all currents are FP64.
template <int P, typename R>
__global__ __launch_bounds__(256) void k3_particles(Mesh3 m, Step3 a)
{
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t p = blk * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    unsigned long long pieces = 0, lost_here = 0;
    __shared__ double s_win[kWin3];
    __shared__ double s_hval[kHash3];
    __shared__ int s_hkey[kHash3];
    __shared__ int s_base;
    const int64_t n = a.stride;
    R *lam = static_cast<R *>(a.lam);
    R *u = static_cast<R *>(a.u);
    // The particle's streams are requested first, so they are in flight
    // while the block sets up its current window.
    uint32_t key = kLost;
    R s0 = R(0), s1 = R(0), s2 = R(0), v0 = R(0), v1 = R(0), v2 = R(0);
    if (p < a.n) {
        key = a.key[p];
        s0 = lam[p];
        s1 = lam[n + p];
        s2 = lam[2 * n + p];
        v0 = u[p];
        v1 = u[n + p];
        v2 = u[2 * n + p];
    }
    for (int j = threadIdx.x; j < kWin3; j += blockDim.x) s_win[j] = 0.0;
    for (int j = threadIdx.x; j < kHash3; j += blockDim.x) {
        s_hkey[j] = -1;
        s_hval[j] = 0.0;
    }
    if (threadIdx.x == 0) {
        // home: the tetrahedron of the block's first particle (thread 0's
        // own, read before any thread of the block writes its key)
        const int home = key == kLost ? 0 : int(key & kTetMask);
        s_base = int(m.tet_ebase[home]) - kBack3;
    }
    __syncthreads();
    const Window3 win{s_win, s_hkey, s_hval, a.cur, s_base};
    const R *rec = static_cast<const R *>(a.rec);
    const R *grad = static_cast<const R *>(sizeof(R) == 4 ? static_cast<const void *>(m.grad32)
                                                          : static_cast<const void *>(m.grad));

    // ---- phase A
    bool moving = false;
    int t = 0, r = 0;
    double L[4] = {0.0, 0.0, 0.0, 0.0};
    R rx = R(0), ry = R(0), rz = R(0);
    if (p < a.n) {
        if (key != kLost) {
            t = int(key & kTetMask);
            r = int(key >> 30);
            unpack_lambda(r, double(s0), double(s1), double(s2), L);
            const R *rc = rec + size_t(kRec) * t;
            V3<R> E{R(0), R(0), R(0)}, B{R(0), R(0), R(0)};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const R lk = R(L[k]);
                E = E + lk * V3<R>{rc[3 * k], rc[3 * k + 1], rc[3 * k + 2]};
                B = B + lk * V3<R>{rc[12 + 3 * k], rc[13 + 3 * k], rc[14 + 3 * k]};
            }
            if (a.b_ext)
                B = B + V3<R>{R(a.b_ext[3 * t]), R(a.b_ext[3 * t + 1]), R(a.b_ext[3 * t + 2])};
            const V3<R> u0{v0, v1, v2};
            const R al = R(a.alpha);
            const V3<R> u1 = push3<P, R>(u0, al * E, al * B, R(a.c), R(a.inv_c2));
            u[p] = u1.x;
            u[n + p] = u1.y;
            u[2 * n + p] = u1.z;
            if (isfinite(u1.x) && isfinite(u1.y) && isfinite(u1.z)) {
                moving = a.cap > 0;
                const R g = gam(u1, R(a.inv_c2));
                const R dt = R(a.dt);
                rx = dt * u1.x / g;
                ry = dt * u1.y / g;
                rz = dt * u1.z / g;
            } else {
                // a bad particle is left where it is
                atomicOr(a.counters + 2, 2ull);
                atomicMin(a.counters + 3, (unsigned long long)p);
            }
        }
    }
    int t0 = -1, bits0 = 0, entry = -1;
    int te0[6] = {0, 0, 0, 0, 0, 0};
    double c[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    bool more = false;  // crossed a face into a neighbour: continue in phase B
    if (moving) {
        t0 = t;
        const int32_t *te = m.tet_edge + 8 * size_t(t);
#pragma unroll
        for (int k = 0; k < 6; ++k) te0[k] = te[k];
        bits0 = te[6];
        R dL[4];
        int ks;
        R ts;
        exit_face(grad + 12 * size_t(t), rx, ry, rz, L, -1, dL, ks, ts);
        ++pieces;
        double Lf[4];
        if (ks < 0 || ts >= R(1)) {
            const int i1 = (r + 1) & 3, i2 = (r + 2) & 3, i3 = (r + 3) & 3;
            const R f1 = R(pick4(L, i1)) + pickR(dL, i1);
            const R f2 = R(pick4(L, i2)) + pickR(dL, i2);
            const R f3 = R(pick4(L, i3)) + pickR(dL, i3);
            unpack_lambda(r, double(f1), double(f2), double(f3), Lf);
            piece_weights(L, Lf, c);
            a.key[p] = uint32_t(t) | (uint32_t(r) << 30);
            lam[p] = f1;
            lam[n + p] = f2;
            lam[2 * n + p] = f3;
        } else {
            const int kp = (ks + 1) & 3, kq = (ks + 2) & 3, kw = (ks + 3) & 3;
            const R lp = R(pick4(L, kp)) + ts * pickR(dL, kp);
            const R lq = R(pick4(L, kq)) + ts * pickR(dL, kq);
            const double lw = (1.0 - double(lp)) - double(lq);
            Lf[0] = Lf[1] = Lf[2] = Lf[3] = 0.0;
            put4(Lf, kp, double(lp));
            put4(Lf, kq, double(lq));
            put4(Lf, kw, lw);
            piece_weights(L, Lf, c);
            const int4 nb4 = m.tet_nbr[t];
            const int nb = ks == 0 ? nb4.x : ks == 1 ? nb4.y : ks == 2 ? nb4.z : nb4.w;
            if (nb < 0) {
                // wall: removed after depositing up to it
                a.key[p] = kLost;
                ++lost_here;
            } else {
                const uint32_t mp = (m.tet_map[t] >> (8 * ks)) & 0xFFu;
                L[0] = L[1] = L[2] = L[3] = 0.0;
                put4(L, int(mp & 3), double(lp));
                put4(L, int((mp >> 2) & 3), double(lq));
                put4(L, int((mp >> 4) & 3), lw);
                r = int((mp >> 4) & 3);
                entry = int(mp >> 6);
                t = nb;
                const R sc = R(1) - ts;
                rx *= sc;
                ry *= sc;
                rz *= sc;
                more = true;
            }
        }
    }

    // ---- first-piece currents: wavefront sum over runs of equal start
    // tetrahedron, then the run's last lane adds them to the window
    {
        const int kprev = __shfl_up(t0, 1, 64);
        const bool head = lane == 0 || kprev != t0;
        const unsigned long long hm = __ballot(head);
        const unsigned long long below = hm & ((2ull << lane) - 1ull);
        const int seg_start = 63 - __clzll(below);
        wave_segmented_sum6(c, lane, seg_start);
        const bool tail = lane == 63 || ((hm >> (lane + 1)) & 1ull);
        if (tail && t0 >= 0)
#pragma unroll
            for (int k = 0; k < 6; ++k)
                win.add(te0[k], (((bits0 >> k) & 1) ? -a.qdt : a.qdt) * c[k]);
    }

    // ---- phase B: the particles that crossed a face
    if (more) continue_move<R>(m, a, win, grad, p, t, r, entry, L, rx, ry, rz, pieces, lost_here);

    // flush the window and the table (non-zero entries hold valid edge ids)
    __syncthreads();
    for (int j = threadIdx.x; j < kWin3; j += blockDim.x) {
        const double v = s_win[j];
        if (v != 0.0) atomic_add_f64(a.cur + (win.base + j), v);
    }
    for (int j = threadIdx.x; j < kHash3; j += blockDim.x) {
        const int k = s_hkey[j];
        const double v = s_hval[j];
        if (k >= 0 && v != 0.0) atomic_add_f64(a.cur + k, v);
    }
    // block totals of pieces and removed particles
    __shared__ unsigned long long s_pc[4], s_lc[4];
    for (int off = 32; off > 0; off >>= 1) {
        pieces += __shfl_down(pieces, off, 64);
        lost_here += __shfl_down(lost_here, off, 64);
    }
    const int wv = threadIdx.x >> 6;
    if (lane == 0) {
        s_pc[wv] = pieces;
        s_lc[wv] = lost_here;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long sp = 0, sl = 0;
        for (int i = 0; i < int(blockDim.x >> 6); ++i) {
            sp += s_pc[i];
            sl += s_lc[i];
        }
        if (sp) atomicAdd(a.counters + 0, sp);
        if (sl) atomicAdd(a.counters + 1, sl);
    }
}

// Sparse products in sliced-ELL form: slices of 64 consecutive rows, each
// stored column-major with the slice's widest row as width (padding: value
// 0, column = the row itself), so a wavefront reads every entry once,
// coalesced.  Each row sums its entries in its stored order.
__global__ __launch_bounds__(256) void k3_hnu(int nf, const int32_t *__restrict__ sptr,
                                              const int32_t *__restrict__ sw,
                                              const int32_t *__restrict__ col,
                                              const double *__restrict__ val,
                                              const double *__restrict__ b, double *__restrict__ h)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    const int sl = f >> 6, lane = f & 63;
    const int w = sw[sl];
    const int64_t base = int64_t(sptr[sl]) + lane;
    double acc = 0.0;
    for (int j = 0; j < w; ++j) acc += val[base + 64 * j] * b[col[base + 64 * j]];
    h[f] = acc;
}

// d += dt (C^T h - i) on free edges (C^T h summed over the edge's faces in
// increasing face order; sign in bit 31 of ef_face), then the current is
// kept for diagnostics and cleared.
__global__ __launch_bounds__(256) void k3_ampere(int ne, const int32_t *__restrict__ ef_ptr,
                                                 const int32_t *__restrict__ ef_face,
                                                 const uint8_t *__restrict__ edge_free,
                                                 const double *__restrict__ h,
                                                 double *__restrict__ cur,
                                                 double *__restrict__ cur_last,
                                                 double *__restrict__ d, double dt)
{
    const int ed = blockIdx.x * blockDim.x + threadIdx.x;
    if (ed >= ne) return;
    double acc = 0.0;
    for (int j = ef_ptr[ed]; j < ef_ptr[ed + 1]; ++j) {
        const int32_t v = ef_face[j];
        const double hv = h[v & 0x7FFFFFFF];
        acc = acc + (v < 0 ? -hv : hv);
    }
    const double i = cur[ed];
    d[ed] = edge_free[ed] ? d[ed] + dt * (acc - i) : 0.0;
    cur_last[ed] = i;
    cur[ed] = 0.0;
}

__global__ __launch_bounds__(256) void k3_spmv(int ne, const int32_t *__restrict__ sptr,
                                               const int32_t *__restrict__ sw,
                                               const int32_t *__restrict__ col,
                                               const double *__restrict__ val,
                                               const uint8_t *__restrict__ edge_free,
                                               const double *__restrict__ d,
                                               double *__restrict__ e)
{
    const int ed = blockIdx.x * blockDim.x + threadIdx.x;
    if (ed >= ne) return;
    const int sl = ed >> 6, lane = ed & 63;
    const int w = sw[sl];
    const int64_t base = int64_t(sptr[sl]) + lane;
    double acc = 0.0;
    if (edge_free[ed])
        for (int j = 0; j < w; ++j) acc += val[base + 64 * j] * d[col[base + 64 * j]];
    e[ed] = acc;
}

// Counting sort by tetrahedron, aggregated per block of kSortB3 particles.
// The particles were sorted at the last sort and have moved a few
// tetrahedra since, so a block's tetrahedra mostly lie in a window of
// kSortBins3 ids placed kSortBack3 below the tetrahedron of its first
// particle: those are counted and placed through LDS (one global atomic per
// touched tetrahedron), the others one by one.
__device__ __forceinline__ uint32_t sort_window3(const Sort3 &a, int64_t b0)
{
    const uint32_t k = a.key_in[b0];
    const uint32_t h = k == kLost ? 0u : (k & kTetMask);
    return h > uint32_t(kSortBack3) ? h - uint32_t(kSortBack3) : 0u;
}

__global__ __launch_bounds__(256) void k3_sort_count(Sort3 a)
{
    __shared__ int32_t h[kSortBins3];
    for (int t = threadIdx.x; t < kSortBins3; t += 256) h[t] = 0;
    const int64_t b0 = int64_t(blockIdx.x) * kSortB3;
    const uint32_t wb = sort_window3(a, b0);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortB3 / 256; ++j) {
        const int64_t i = b0 + j * 256 + int(threadIdx.x);
        const uint32_t k = i < a.n ? a.key_in[i] : kLost;
        if (k == kLost) continue;
        const uint32_t f = k & kTetMask, bin = f - wb;
        if (bin < uint32_t(kSortBins3))
            atomicAdd(&h[bin], 1);
        else
            atomicAdd(a.counts + f, 1);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kSortBins3; t += 256)
        if (h[t]) atomicAdd(a.counts + wb + uint32_t(t), h[t]);
}

// ... exclusive scan of counts[0..nt] into cursor: each block of 1024
// scans its chunk and reports the chunk total ...
__global__ __launch_bounds__(1024) void k3_scan_chunks(int n, const int32_t *__restrict__ counts,
                                                       int32_t *__restrict__ cursor,
                                                       int32_t *__restrict__ chunk_sums)
{
    __shared__ int32_t part[1024];
    const int i = blockIdx.x * 1024 + threadIdx.x;
    const int32_t v = i < n ? counts[i] : 0;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int32_t x = threadIdx.x >= unsigned(off) ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += x;
        __syncthreads();
    }
    if (i < n) cursor[i] = part[threadIdx.x] - v;
    if (threadIdx.x == 1023) chunk_sums[blockIdx.x] = part[1023];
}

// ... the chunk totals are scanned by one block (sequential runs per
// thread, so any number of chunks fits) ...
__global__ __launch_bounds__(1024) void k3_scan_totals(int nchunk, int32_t *__restrict__ sums)
{
    __shared__ int32_t part[1024];
    const int tid = threadIdx.x;
    const int per = (nchunk + 1023) / 1024;
    const int lo = min(nchunk, tid * per), hi = min(nchunk, lo + per);
    int32_t s = 0;
    for (int i = lo; i < hi; ++i) s += sums[i];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int32_t x = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += x;
        __syncthreads();
    }
    int32_t run = part[tid] - s;
    for (int i = lo; i < hi; ++i) {
        const int32_t c = sums[i];
        sums[i] = run;
        run += c;
    }
}

// ... and added back to every chunk.
__global__ __launch_bounds__(1024) void k3_scan_add(int n, int32_t *__restrict__ cursor,
                                                    const int32_t *__restrict__ sums)
{
    const int i = blockIdx.x * 1024 + threadIdx.x;
    if (i < n) cursor[i] += sums[blockIdx.x];
}

// ... then scatter: every block ranks its particles inside their window
// bins, reserves each touched tetrahedron's places with one atomic, and
// writes, in destination order through an LDS permutation, the input index
// of each place (particles outside the window reserve their place alone).
// Only this 4-byte index is scattered: particles that moved to a
// neighbouring tetrahedron land a few at a time in many places, and each
// such write fills part of a line ...
__global__ __launch_bounds__(256) void k3_sort_scatter(Sort3 a)
{
    __shared__ int32_t cnt[kSortBins3];  // count per bin, then its global base
    __shared__ int32_t loc[kSortBins3];  // exclusive offset of the bin inside the block
    __shared__ int32_t wsum[4];
    __shared__ int32_t n_in, n_out;
    __shared__ uint16_t s_src[kSortB3];  // block slot -> block-local input index
    __shared__ int32_t s_dst[kSortB3];   // block slot -> destination
    constexpr int kPer = kSortB3 / 256;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int t = tid; t < kSortBins3; t += 256) cnt[t] = 0;
    if (tid == 0) n_out = 0;
    const int64_t b0 = int64_t(blockIdx.x) * kSortB3;
    const uint32_t wb = sort_window3(a, b0);
    __syncthreads();
    int32_t bin[kPer], rank[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int64_t i = b0 + j * 256 + tid;
        const uint32_t k = i < a.n ? a.key_in[i] : kLost;
        bin[j] = -1;
        rank[j] = -1;
        if (k == kLost) continue;
        const uint32_t f = k & kTetMask, b = f - wb;
        if (b < uint32_t(kSortBins3)) {
            bin[j] = int32_t(b);
            rank[j] = atomicAdd(&cnt[b], 1);
        } else {
            // outside the window: its own place, kept at the end of the block slots
            const int r = atomicAdd(&n_out, 1);
            s_dst[kSortB3 - 1 - r] = atomicAdd(a.cursor + f, 1);
            s_src[kSortB3 - 1 - r] = uint16_t(j * 256 + tid);
        }
    }
    __syncthreads();
    // exclusive scan of the bin counts (kSortBins3 / 256 per thread)
    constexpr int kBpt = kSortBins3 / 256;
    int32_t cq[kBpt], run = 0;
#pragma unroll
    for (int q = 0; q < kBpt; ++q) {
        cq[q] = cnt[kBpt * tid + q];
        run += cq[q];
    }
    int32_t incl = run;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int32_t before = incl - run;
    for (int w = 0; w < wv; ++w) before += wsum[w];
    if (tid == 255) n_in = before + run;
#pragma unroll
    for (int q = 0; q < kBpt; ++q) {
        loc[kBpt * tid + q] = before;
        // one global reservation per touched tetrahedron
        const int32_t g = cq[q] ? atomicAdd(a.cursor + wb + uint32_t(kBpt * tid + q), cq[q]) : 0;
        cnt[kBpt * tid + q] = g;
        before += cq[q];
    }
    __syncthreads();
    // block slots of the in-window particles: bin offset + rank
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        if (bin[j] < 0) continue;
        const int slot = loc[bin[j]] + rank[j];
        s_src[slot] = uint16_t(j * 256 + tid);
        s_dst[slot] = cnt[bin[j]] + rank[j];
    }
    __syncthreads();
    const int nin = n_in, nout = n_out;
    for (int s = tid; s < kSortB3; s += 256) {
        if (s >= nin && s < kSortB3 - nout) continue;
        a.perm[s_dst[s]] = int32_t(b0 + s_src[s]);
    }
}

// ... and every output slot below the live total gathers its particle:
// the writes are sequential and the reads come from nearby slots of the
// nearly sorted input.
template <typename R>
__global__ __launch_bounds__(256) void k3_sort_gather(Sort3 a)
{
    const int64_t q = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (q >= int64_t(a.cursor[a.nt])) return;
    const int64_t i = a.perm[q];
    const R *li = static_cast<const R *>(a.lam_in), *ui = static_cast<const R *>(a.u_in);
    R *lo = static_cast<R *>(a.lam_out), *uo = static_cast<R *>(a.u_out);
    a.key_out[q] = a.key_in[i];
    a.pid_out[q] = a.pid_in[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        lo[c * a.stride_out + q] = li[c * a.stride_in + i];
        uo[c * a.stride_out + q] = ui[c * a.stride_in + i];
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k3_charge(int64_t n, const uint32_t *__restrict__ key,
                                                 const R *__restrict__ lam, int64_t stride,
                                                 const int4 *__restrict__ tet_node, double qw,
                                                 double *__restrict__ q)
{
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t k = key[p];
    if (k == kLost) return;
    double L[4];
    unpack_lambda(int(k >> 30), double(lam[p]), double(lam[stride + p]), double(lam[2 * stride + p]),
                  L);
    const int4 tn = tet_node[k & kTetMask];
    atomic_add_f64(q + tn.x, qw * L[0]);
    atomic_add_f64(q + tn.y, qw * L[1]);
    atomic_add_f64(q + tn.z, qw * L[2]);
    atomic_add_f64(q + tn.w, qw * L[3]);
}

__global__ __launch_bounds__(256) void k3_divd(int ne, const int2 *__restrict__ edge_nodes,
                                               const double *__restrict__ d,
                                               double *__restrict__ out)
{
    const int ed = blockIdx.x * blockDim.x + threadIdx.x;
    if (ed >= ne) return;
    const int2 en = edge_nodes[ed];
    atomic_add_f64(out + en.x, d[ed]);
    atomic_add_f64(out + en.y, -d[ed]);
}

__global__ __launch_bounds__(256) void k3_divb(int nt, const int4 *__restrict__ tet_face,
                                               const int32_t *__restrict__ fout_bits,
                                               const double *__restrict__ b,
                                               double *__restrict__ out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const int4 f = tet_face[t];
    const int bits = fout_bits[t];
    const double v0 = (bits & 1) ? -b[f.x] : b[f.x];
    const double v1 = (bits & 2) ? -b[f.y] : b[f.y];
    const double v2 = (bits & 4) ? -b[f.z] : b[f.z];
    const double v3 = (bits & 8) ? -b[f.w] : b[f.w];
    out[t] = ((v0 + v1) + v2) + v3;
}

}  // namespace

hipError_t launch3_faraday(hipStream_t s, int nf, const int4 *face_edge, const double *e,
                           double *b, double *bavg, double dt)
{
    if (nf <= 0) return hipSuccess;
    FETD_LAUNCH(k3_faraday, dim3(grid_for(nf, 256)), dim3(256), 0, s, nf, face_edge, e, b,
                       bavg, dt);
    return hipGetLastError();
}

hipError_t launch3_record(hipStream_t s, int nt, const Mesh3 &m, const double *e,
                          const double *e_ext, const double *bavg, void *rec, bool fp32)
{
    if (nt <= 0) return hipSuccess;
    if (fp32)
        FETD_LAUNCH(k3_record<float>, dim3(grid_for(nt, 256)), dim3(256), 0, s, nt, m, e,
                           e_ext, bavg, static_cast<float *>(rec));
    else
        FETD_LAUNCH(k3_record<double>, dim3(grid_for(nt, 256)), dim3(256), 0, s, nt, m, e,
                           e_ext, bavg, static_cast<double *>(rec));
    return hipGetLastError();
}

template <typename R>
void launch3_particles_t(hipStream_t s, const Mesh3 &m, const Step3 &a, int pusher)
{
    const dim3 grid(grid_for(a.n, kBlock)), block(kBlock);
    switch (pusher) {
    case 0: FETD_LAUNCH((k3_particles<0, R>), grid, block, 0, s, m, a); break;
    case 1: FETD_LAUNCH((k3_particles<1, R>), grid, block, 0, s, m, a); break;
    case 2: FETD_LAUNCH((k3_particles<2, R>), grid, block, 0, s, m, a); break;
    default: FETD_LAUNCH((k3_particles<3, R>), grid, block, 0, s, m, a); break;
    }
}

hipError_t launch3_particles(hipStream_t s, const Mesh3 &m, const Step3 &a, int pusher, bool fp32)
{
    if (a.n <= 0) return hipSuccess;
    if (fp32)
        launch3_particles_t<float>(s, m, a, pusher);
    else
        launch3_particles_t<double>(s, m, a, pusher);
    return hipGetLastError();
}

hipError_t launch3_hnu(hipStream_t s, int nf, const Sell &m, const double *b, double *h)
{
    if (nf <= 0) return hipSuccess;
    FETD_LAUNCH(k3_hnu, dim3(grid_for(nf, 256)), dim3(256), 0, s, nf, m.sptr, m.sw, m.col,
                       m.val, b, h);
    return hipGetLastError();
}

hipError_t launch3_ampere(hipStream_t s, int ne, const int32_t *ef_ptr, const int32_t *ef_face,
                          const uint8_t *edge_free, const double *h, double *cur,
                          double *cur_last, double *d, double dt)
{
    if (ne <= 0) return hipSuccess;
    FETD_LAUNCH(k3_ampere, dim3(grid_for(ne, 256)), dim3(256), 0, s, ne, ef_ptr, ef_face,
                       edge_free, h, cur, cur_last, d, dt);
    return hipGetLastError();
}

hipError_t launch3_spmv(hipStream_t s, int ne, const Sell &m, const uint8_t *edge_free,
                        const double *d, double *e)
{
    if (ne <= 0) return hipSuccess;
    FETD_LAUNCH(k3_spmv, dim3(grid_for(ne, 256)), dim3(256), 0, s, ne, m.sptr, m.sw, m.col,
                       m.val, edge_free, d, e);
    return hipGetLastError();
}

hipError_t launch3_sort(hipStream_t s, const Sort3 &a)
{
    if (a.n <= 0) return hipSuccess;
    hipError_t e = hipMemsetAsync(a.counts, 0, sizeof(int32_t) * (size_t(a.nt) + 1), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k3_sort_count, dim3(grid_for(a.n, kSortB3)), dim3(256), 0, s, a);
    const int n1 = a.nt + 1, nchunk = (n1 + 1023) / 1024;
    hipLaunchKernelGGL(k3_scan_chunks, dim3(nchunk), dim3(1024), 0, s, n1, a.counts, a.cursor,
                       a.chunk_sums);
    hipLaunchKernelGGL(k3_scan_totals, dim3(1), dim3(1024), 0, s, nchunk, a.chunk_sums);
    hipLaunchKernelGGL(k3_scan_add, dim3(nchunk), dim3(1024), 0, s, n1, a.cursor, a.chunk_sums);
    hipLaunchKernelGGL(k3_sort_scatter, dim3(grid_for(a.n, kSortB3)), dim3(256), 0, s, a);
    if (a.elem_bytes == 4)
        hipLaunchKernelGGL(k3_sort_gather<float>, dim3(grid_for(a.n, 256)), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k3_sort_gather<double>, dim3(grid_for(a.n, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch3_charge(hipStream_t s, int64_t n, const uint32_t *key, const void *lam,
                          bool fp32, int64_t stride, const int4 *tet_node, double qw, double *q)
{
    if (n <= 0) return hipSuccess;
    if (fp32)
        hipLaunchKernelGGL(k3_charge<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, n, key,
                           static_cast<const float *>(lam), stride, tet_node, qw, q);
    else
        hipLaunchKernelGGL(k3_charge<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, n, key,
                           static_cast<const double *>(lam), stride, tet_node, qw, q);
    return hipGetLastError();
}

hipError_t launch3_divd(hipStream_t s, int ne, const int2 *edge_nodes, const double *d,
                        double *out)
{
    if (ne <= 0) return hipSuccess;
    hipLaunchKernelGGL(k3_divd, dim3(grid_for(ne, 256)), dim3(256), 0, s, ne, edge_nodes, d, out);
    return hipGetLastError();
}

hipError_t launch3_divb(hipStream_t s, int nt, const int4 *tet_face, const int32_t *fout_bits,
                        const double *b, double *out)
{
    if (nt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k3_divb, dim3(grid_for(nt, 256)), dim3(256), 0, s, nt, tet_face, fout_bits,
                       b, out);
    return hipGetLastError();
}

}  // namespace fetd3
