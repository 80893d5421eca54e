// HIP kernels (gfx950) of the charge-conserving relativistic FETD-PIC step.
//
// Method: arXiv:1707.04333 (Na, Moon, Omelchenko, Teixeira).  One step:
//   k_faraday        b^{n+1/2} = b^{n-1/2} - dt C e^n (Sec. II.A eq.
//                    semi.dis.curl.1), B^n = (B^{n+1/2} + B^{n-1/2})/2 (Sec.
//                    II.C) and the per-triangle gather record of e^n;
//   k_particle_step  gather (Sec. II.B), push (Sec. II.C), move and track,
//                    scatter of the exact W1 line-integral current (Sec.
//                    II.D eq. I.assign), fused per particle;
//   k_ampere         d += dt (C^T [*mu^-1] b^{n+1/2} - i^{n+1/2})
//                    (Sec. II.A eq. semi.dis.curl.2 in the d = [*eps] e form);
//   k_spmv           e^{n+1} = M~ d^{n+1} with the sparse approximate inverse.
// Nothing here is a dense contraction: the kernels are bandwidth kernels
// (coalesced SoA particle streams, per-triangle tables read through the
// cache, FP64 current reduced within each wavefront before the atomics).
#include "fetd_internal.h"
#include "stage_events.h"

#include <hip/hip_runtime.h>

namespace fetd {
namespace {

template <typename R>
struct Vec2;
template <>
struct Vec2<float> {
    using type = float2;
};
template <>
struct Vec2<double> {
    using type = double2;
};

// Three values addressed by a run-time local index without spilling to
// scratch memory (selects instead of an indexed array).
template <typename T>
struct Tri3 {
    T v0, v1, v2;
    __device__ __forceinline__ T get(int i) const { return i == 0 ? v0 : (i == 1 ? v1 : v2); }
    __device__ __forceinline__ void set(int i, T x)
    {
        v0 = (i == 0) ? x : v0;
        v1 = (i == 1) ? x : v1;
        v2 = (i == 2) ? x : v2;
    }
};

__device__ __forceinline__ int next3(int i) { return i == 2 ? 0 : i + 1; }
__device__ __forceinline__ int prev3(int i) { return i == 0 ? 2 : i - 1; }

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous run of tiles so the per-triangle tables a tile touches stay
// in one XCD's L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb)
{
    const int64_t x = b & 7, j = b >> 3;
    const int64_t per = nb >> 3, rem = nb & 7;
    return x < rem ? x * (per + 1) + j : rem * (per + 1) + (x - rem) * per + j;
}

__device__ __forceinline__ void atomic_add_f64(double *p, double v) { unsafeAtomicAdd(p, v); }

// Reciprocal and reciprocal square root: the hardware approximations
// (about 1 ulp) in FP32, IEEE-rounded division and square root in FP64.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }

// Cross-lane move of a double by a DPP control; lanes whose source is
// outside the row (or rows disabled by RM) read 0.
template <int CTRL, int RM>
__device__ __forceinline__ double dpp_f64(double v)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, RM, 0xF, true);
    hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, RM, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Inclusive segmented sum over the wavefront: every lane ends with the sum
// of its run [seg_start, lane].  Row shifts 1, 2, 4, 8 inside each row of
// 16 lanes, then the row-15 and row-31 broadcasts across rows.
template <int CTRL, int RM>
__device__ __forceinline__ void seg_step(double &c0, double &c1, double &c2, bool take)
{
    const double o0 = dpp_f64<CTRL, RM>(c0);
    const double o1 = dpp_f64<CTRL, RM>(c1);
    const double o2 = dpp_f64<CTRL, RM>(c2);
    if (take) {
        c0 += o0;
        c1 += o1;
        c2 += o2;
    }
}

__device__ __forceinline__ void wave_segmented_sum(double &c0, double &c1, double &c2, int lane,
                                                   int seg_start)
{
    const int in_row = lane & 15;
    seg_step<0x111, 0xF>(c0, c1, c2, in_row >= 1 && lane - 1 >= seg_start);
    seg_step<0x112, 0xF>(c0, c1, c2, in_row >= 2 && lane - 2 >= seg_start);
    seg_step<0x114, 0xF>(c0, c1, c2, in_row >= 4 && lane - 4 >= seg_start);
    seg_step<0x118, 0xF>(c0, c1, c2, in_row >= 8 && lane - 8 >= seg_start);
    seg_step<0x142, 0xA>(c0, c1, c2, (lane & 16) && (lane & ~15) - 1 >= seg_start);
    seg_step<0x143, 0xC>(c0, c1, c2, lane >= 32 && 31 >= seg_start);
}

// ---------------------------------------------------------------------
// Pushers (Sec. II.C), specialised to in-plane u and E with B along z.
// eps = alpha E, bz = alpha Bz (beta), all in the precision R.
// ---------------------------------------------------------------------
template <int P, typename R>
__device__ __forceinline__ void push2(R &ux, R &uy, R ex, R ey, R bz, R inv_c2)
{
    const R one = R(1);
    if constexpr (P == 2) {
        // Vay: exact solution of u+ = u' + (u+/gamma+) x beta with
        // u' = u + 2 eps + v(u) x beta.
        const R rg0 = rsqrt_(one + (ux * ux + uy * uy) * inv_c2);
        const R vx = ux * rg0, vy = uy * rg0;
        const R upx = ux + ex + vy * bz + ex;
        const R upy = uy + ey - vx * bz + ey;
        const R gp2 = one + (upx * upx + upy * upy) * inv_c2;
        const R bb = bz * bz;
        const R sig = gp2 - bb;
        const R gn = sqrt_(R(0.5) * (sig + sqrt_(sig * sig + R(4) * bb)));
        const R tz = bz * rcp(gn);
        const R s = rcp(one + tz * tz);
        ux = s * (upx + upy * tz);
        uy = s * (upy - upx * tz);
        return;
    }
    const R umx = ux + ex, umy = uy + ey;
    const R gm2 = one + (umx * umx + umy * umy) * inv_c2;
    R tz;
    if constexpr (P == 3) {
        // Higuera-Cary: gamma of the midpoint momentum.
        const R bb = bz * bz;
        const R sig = gm2 - bb;
        const R gh = sqrt_(R(0.5) * (sig + sqrt_(sig * sig + R(4) * bb)));
        tz = bz * rcp(gh);
    } else if constexpr (P == 1) {
        // Boris with the tan correction: t = (beta/|beta|) tan(|beta|/gbar).
        tz = tan(bz * rsqrt_(gm2));
    } else {
        tz = bz * rsqrt_(gm2);
    }
    const R sz = R(2) * tz * rcp(one + tz * tz);
    const R qx = umx + umy * tz;   // u' = u- + u- x t
    const R qy = umy - umx * tz;
    ux = umx + qy * sz + ex;       // u+ = u- + u' x s, then the second half kick
    uy = umy - qx * sz + ey;
}

// ---------------------------------------------------------------------
// Block-local FP64 current accumulation: a window of kWin consecutive
// device edge ids in LDS, placed by the tile's home triangle.  Triangle-
// sorted tiles touch a few dozen edges, almost all inside the window; an
// edge outside it (a neighbour far away in the triangle order) goes
// straight to the global accumulator.  Neither path waits for a result.
// ---------------------------------------------------------------------
struct LdsCurrent {
    double *acc;     // [kWin]
    double *global;  // current accumulator of the step
    uint32_t base;   // first edge id of the window

    __device__ __forceinline__ void add(int edge, double v) const
    {
        const uint32_t j = uint32_t(edge) - base;
        if (j < uint32_t(kWin))
            __hip_atomic_fetch_add(acc + j, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else
            atomic_add_f64(global + edge, v);
    }
};

// ---------------------------------------------------------------------
// Typed access to the per-triangle tables and particle streams with 32-bit
// byte offsets (scalar base + vector offset addressing).
// ---------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T ld(const void *base, uint32_t off)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off);
}
template <typename T>
__device__ __forceinline__ void st(void *base, uint32_t off, T v)
{
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off) = v;
}

template <typename R>
struct Rec {
    R v0x, v0y, v1x, v1y, v2x, v2y, bz;
};
__device__ __forceinline__ Rec<float> load_rec(const void *rec, uint32_t f)
{
    const float4 a = ld<float4>(rec, f * 32u), b = ld<float4>(rec, f * 32u + 16u);
    return {a.x, a.y, a.z, a.w, b.x, b.y, b.z};
}
__device__ __forceinline__ Rec<double> load_rec64(const void *rec, uint32_t f)
{
    const double2 a = ld<double2>(rec, f * 64u), b = ld<double2>(rec, f * 64u + 16u);
    const double2 c = ld<double2>(rec, f * 64u + 32u), d = ld<double2>(rec, f * 64u + 48u);
    return {a.x, a.y, b.x, b.y, c.x, c.y, d.x};
}

template <typename R>
struct Grad {
    R x0, y0, x1, y1, x2, y2;
};
__device__ __forceinline__ Grad<float> load_grad(const MeshView &m, uint32_t f, float)
{
    const float4 a = ld<float4>(m.grad32, f * 32u), b = ld<float4>(m.grad32, f * 32u + 16u);
    return {a.x, a.y, a.z, a.w, b.x, b.y};
}
__device__ __forceinline__ Grad<double> load_grad(const MeshView &m, uint32_t f, double)
{
    const double2 a = ld<double2>(m.grad64, f * 48u), b = ld<double2>(m.grad64, f * 48u + 16u);
    const double2 c = ld<double2>(m.grad64, f * 48u + 32u);
    return {a.x, a.y, b.x, b.y, c.x, c.y};
}

// x_i for a run-time local index i (two selects).
template <typename T>
__device__ __forceinline__ T pick(int i, T x0, T x1, T x2)
{
    return i == 0 ? x0 : (i == 1 ? x1 : x2);
}

// Exit edge of a straight move inside a triangle (the tracking rule):
// candidates are the local edges k with dL_k < 0 other than the entry edge,
// tau_k = max(l_k, 0) / (-dL_k), the smallest tau wins, ties to the
// smallest k.  Branch-free.
template <typename R>
__device__ __forceinline__ void exit_edge(R l0, R l1, R l2, R d0, R d1, R d2, int entry, int &ks,
                                          R &ts)
{
    const bool h0 = entry != 0 && d0 < R(0);
    const bool h1 = entry != 1 && d1 < R(0);
    const bool h2 = entry != 2 && d2 < R(0);
    const R t0 = (l0 > R(0) ? l0 : R(0)) * rcp(-d0);
    const R t1 = (l1 > R(0) ? l1 : R(0)) * rcp(-d1);
    const R t2 = (l2 > R(0) ? l2 : R(0)) * rcp(-d2);
    ks = h0 ? 0 : -1;
    ts = h0 ? t0 : R(0);
    const bool b1 = h1 && (ks < 0 || t1 < ts);
    ks = b1 ? 1 : ks;
    ts = b1 ? t1 : ts;
    const bool b2 = h2 && (ks < 0 || t2 < ts);
    ks = b2 ? 2 : ks;
    ts = b2 ? t2 : ts;
}

// One straight piece inside triangle f.  Given the start barycentrics (L in
// the tracking precision, Ls in FP64), the move (rx, ry) and the entry
// edge, decide the exit and produce the end point of the piece (Lf, FP64)
// and its current cross terms w_k = Ls_a Lf_b - Lf_a Ls_b (eq. I.assign,
// (a, b) = (k+1, k+2)).  When the piece ends inside f, L is advanced to
// the end point (the stored pair is L at the two non-derived slots).
template <typename R>
struct Piece {
    int ks;     // exit edge, or -1
    R ts;       // exit parameter
    R la;       // l_{ks+1} at the exit point
    bool done;  // ends inside f
    double w0, w1, w2;
};

template <typename R>
__device__ __forceinline__ Piece<R> trace_piece(const Grad<R> &g, R &l0, R &l1, R &l2,
                                                double s0, double s1, double s2, int r, R rx,
                                                R ry, int entry)
{
    Piece<R> pc;
    const R d0 = g.x0 * rx + g.y0 * ry;
    const R d1 = g.x1 * rx + g.y1 * ry;
    const R d2 = g.x2 * rx + g.y2 * ry;
    exit_edge(l0, l1, l2, d0, d1, d2, entry, pc.ks, pc.ts);
    pc.done = pc.ks < 0 || pc.ts >= R(1);
    // end inside: every coordinate advanced, the derived slot re-derived in FP64
    const R n0 = l0 + d0, n1 = l1 + d1, n2 = l2 + d2;
    const int rp = next3(r), rq = prev3(r);
    const double dp = double(pick(rp, n0, n1, n2)), dq = double(pick(rq, n0, n1, n2));
    const double dr = (1.0 - dp) - dq;
    double e0 = r == 0 ? dr : double(n0);
    double e1 = r == 1 ? dr : double(n1);
    double e2 = r == 2 ? dr : double(n2);
    // exit through edge ks: l_ks = 0, l_a = l_a + ts dL_a, l_b = 1 - l_a
    const int ka = next3(pc.ks < 0 ? 0 : pc.ks);
    pc.la = pick(ka, l0, l1, l2) + pc.ts * pick(ka, d0, d1, d2);
    const double xa = double(pc.la), xb = 1.0 - xa;
    if (!pc.done) {
        e0 = pc.ks == 0 ? 0.0 : (ka == 0 ? xa : xb);
        e1 = pc.ks == 1 ? 0.0 : (ka == 1 ? xa : xb);
        e2 = pc.ks == 2 ? 0.0 : (ka == 2 ? xa : xb);
    } else {
        l0 = n0;
        l1 = n1;
        l2 = n2;
    }
    pc.w0 = s1 * e2 - e1 * s2;
    pc.w1 = s2 * e0 - e2 * s0;
    pc.w2 = s0 * e1 - e0 * s1;
    return pc;
}

// Continue a particle past the edge it is leaving: it enters triangle nbf
// (-1 = wall) through that triangle's local edge kk at the point where
// l_{kk+2} = la, with the fraction ts of its move done.  Trace and deposit
// piece after piece until the move ends inside a triangle (returns true),
// meets a wall (lost) or exceeds the crossing cap.  The tables of each new
// triangle are loaded together, neighbours included, so every crossing
// costs one round trip to the cache.  On return (f, r, l) hold the end
// triangle, derived slot and barycentrics.
template <typename R>
__device__ __forceinline__ bool continue_track(const MeshView &m, const LdsCurrent &dep, double q,
                                               int cap, uint32_t &f, int &r, int nbf, int kk,
                                               R la, R ts, R &l0, R &l1, R &l2, R rx, R ry,
                                               unsigned long long &nseg, bool &capped)
{
    for (int it = 1;; ++it) {
        if (nbf < 0) return false;  // wall
        if (it >= cap) {
            capped = true;
            return false;
        }
        f = uint32_t(nbf);
        const Grad<R> g = load_grad(m, f, R(0));
        const int4 te = ld<int4>(m.tri_edge, f * 16u);
        const int4 nb = ld<int4>(m.tri_nbr, f * 16u);
        // CCW neighbours traverse the shared edge in opposite directions:
        // node ks+1 of the old triangle is node kk+2 here and vice versa.
        const int b2 = prev3(kk);
        l0 = kk == 0 ? R(0) : (b2 == 0 ? la : R(1) - la);
        l1 = kk == 1 ? R(0) : (b2 == 1 ? la : R(1) - la);
        l2 = kk == 2 ? R(0) : (b2 == 2 ? la : R(1) - la);
        const double xa = double(la), xb = 1.0 - xa;
        const double s0 = kk == 0 ? 0.0 : (b2 == 0 ? xa : xb);
        const double s1 = kk == 1 ? 0.0 : (b2 == 1 ? xa : xb);
        const double s2 = kk == 2 ? 0.0 : (b2 == 2 ? xa : xb);
        r = next3(kk);
        const R sc = R(1) - ts;
        rx = rx * sc;
        ry = ry * sc;
        const Piece<R> pc = trace_piece(g, l0, l1, l2, s0, s1, s2, r, rx, ry, kk);
        nseg += 1;
        dep.add(te.x, ((te.w & 1) ? -q : q) * pc.w0);
        dep.add(te.y, ((te.w & 2) ? -q : q) * pc.w1);
        dep.add(te.z, ((te.w & 4) ? -q : q) * pc.w2);
        if (pc.done) return true;
        nbf = pick(pc.ks, nb.x, nb.y, nb.z);
        kk = (nb.w >> (2 * pc.ks)) & 3;
        la = pc.la;
        ts = pc.ts;
    }
}

// Store the end state of a particle (or mark it lost) and count it.
template <typename R>
__device__ __forceinline__ void finish_particle(const StepArgs &a, uint32_t i, uint32_t f, int r,
                                                R l0, R l1, R l2, bool ok, bool capped,
                                                unsigned long long &nlost)
{
    using R2 = typename Vec2<R>::type;
    uint32_t key = kLost;
    if (capped) {
        atomicOr(a.counters + 2, 1ull);
        atomicMin(a.counters + 3, (unsigned long long)(a.pid ? a.pid[i] : i));
    }
    if (ok) {
        key = f | (uint32_t(r) << 30);
        R2 np2;
        np2.x = pick(next3(r), l0, l1, l2);
        np2.y = pick(prev3(r), l0, l1, l2);
        st<R2>(a.lam, i * uint32_t(sizeof(R2)), np2);
    } else {
        nlost += 1;
    }
    st<uint32_t>(a.key, i * 4u, key);
}

// ---------------------------------------------------------------------
// Fused particle stage.  Each block owns kPPT * kBlock consecutive
// (triangle-sorted) particles.  Phase 1, one particle per thread per pass:
// gather, push, move and the first straight piece (most particles stay in
// their triangle); the particles that leave it are queued in LDS.  Phase 2
// finishes the queued particles with all lanes busy.  Currents go to the
// block's LDS edge table and are flushed once per block.
// ---------------------------------------------------------------------
constexpr int kQueue = 512;

template <typename R>
struct Queue {
    uint32_t idx[kQueue];   // particle index
    uint32_t fk[kQueue];    // triangle | exit edge << 30
    R ts[kQueue], la[kQueue], rx[kQueue], ry[kQueue];
};

template <typename R>
struct TileShared {
    double acc[kWin];
    Queue<R> q;
    int qn;
    unsigned long long red[2][kBlock / 64];
};

// One tile of kPPT * kBlock particles of one species (tile index `tile`
// within the species), processed by the whole block.
template <int P, typename R>
__device__ __forceinline__ void particle_tile(const MeshView &m, const StepArgs &a, uint32_t tile,
                                              TileShared<R> &sh)
{
    using R2 = typename Vec2<R>::type;
    constexpr uint32_t kR2 = sizeof(R2);
    double *s_acc = sh.acc;
    Queue<R> &s_q = sh.q;
    int &s_qn = sh.qn;
    auto &red = sh.red;
    // The particle streams of the next pass are loaded while the current
    // pass computes (unconditionally: the loads never wait for the key).
    uint32_t i_next = tile * kPPT * kBlock + threadIdx.x;
    uint32_t key_next = kLost;
    R2 pr_next{}, uu_next{};
    if (int64_t(i_next) < a.n) {
        key_next = ld<uint32_t>(a.key, i_next * 4u);
        pr_next = ld<R2>(a.lam, i_next * kR2);
        uu_next = ld<R2>(a.u, i_next * kR2);
    }
    uint32_t wbase = 0;
    if (a.tile_home) {
        const uint32_t home = a.tile_home[tile];
        wbase = m.tri_ebase[home > kWinBack ? home - kWinBack : 0u];
    }
    for (int t = threadIdx.x; t < kWin; t += kBlock) s_acc[t] = 0.0;
    if (threadIdx.x == 0) s_qn = 0;
    __syncthreads();
    const LdsCurrent dep{s_acc, a.cur, wbase};
    const int lane = threadIdx.x & 63;
    unsigned long long nseg = 0, nlost = 0;
    const double q = a.qdt;

    for (int pass = 0; pass < kPPT; ++pass) {
        const uint32_t i = i_next;
        const uint32_t key = key_next;
        const R2 pr = pr_next, uu = uu_next;
        const bool alive = key != kLost;
        // Dead lanes (removed particles, tail of the last tile) compute on
        // triangle 0 and store nothing.
        const uint32_t f = alive ? (key & kTriMask) : 0u;
        const int r = alive ? int(key >> 30) : 0;
        // The pass's triangle tables are requested before the next pass's
        // particle streams.
        Rec<R> rc;
        if constexpr (sizeof(R) == 4) rc = load_rec(a.rec, f);
        else rc = load_rec64(a.rec, f);
        const Grad<R> g = load_grad(m, f, R(0));
        const int4 te = ld<int4>(m.tri_edge, f * 16u);
        const int4 nb = ld<int4>(m.tri_nbr, f * 16u);
        if (pass + 1 < kPPT) {
            i_next = i + kBlock;
            key_next = kLost;
            if (int64_t(i_next) < a.n) {
                key_next = ld<uint32_t>(a.key, i_next * 4u);
                pr_next = ld<R2>(a.lam, i_next * kR2);
                uu_next = ld<R2>(a.u, i_next * kR2);
            }
        }

        // local barycentrics: slot r derived from the stored pair
        const R dR = (R(1) - pr.x) - pr.y;
        R l0 = r == 0 ? dR : (r == 1 ? pr.y : pr.x);
        R l1 = r == 0 ? pr.x : (r == 1 ? dR : pr.y);
        R l2 = r == 0 ? pr.y : (r == 1 ? pr.x : dR);
        const double dD = (1.0 - double(pr.x)) - double(pr.y);
        const double s0 = r == 0 ? dD : double(l0);
        const double s1 = r == 1 ? dD : double(l1);
        const double s2 = r == 2 ? dD : double(l2);

        // Gather (Sec. II.B): E = sum_n l_n V_n from the triangle record.
        R ex = l0 * rc.v0x + l1 * rc.v1x + l2 * rc.v2x;
        R ey = l0 * rc.v0y + l1 * rc.v1y + l2 * rc.v2y;
        if (a.has_affine) {
            R x, y;
            if constexpr (sizeof(R) == 4) {
                const float4 va = ld<float4>(m.vxy32, f * 32u), vb = ld<float4>(m.vxy32, f * 32u + 16u);
                x = l0 * va.x + l1 * va.z + l2 * vb.x;
                y = l0 * va.y + l1 * va.w + l2 * vb.y;
            } else {
                const double2 va = ld<double2>(m.vxy64, f * 48u), vb = ld<double2>(m.vxy64, f * 48u + 16u);
                const double2 vc = ld<double2>(m.vxy64, f * 48u + 32u);
                x = l0 * va.x + l1 * vb.x + l2 * vc.x;
                y = l0 * va.y + l1 * vb.y + l2 * vc.y;
            }
            ex += R(a.aff[0]) + R(a.aff[2]) * x + R(a.aff[3]) * y;
            ey += R(a.aff[1]) + R(a.aff[4]) * x + R(a.aff[5]) * y;
        }

        // Push (Sec. II.C).
        const R alpha = R(a.alpha);
        R ux = uu.x, uy = uu.y;
        push2<P, R>(ux, uy, alpha * ex, alpha * ey, alpha * rc.bz, R(a.inv_c2));
        const bool finite = isfinite(ux) && isfinite(uy);
        if (alive) {
            R2 un;
            un.x = ux;
            un.y = uy;
            st<R2>(a.u, i * kR2, un);
        }

        // Move: dr = dt u / gamma (Sec. II.C eq. eq.motion.dis).
        const R ginv = rsqrt_(R(1) + (ux * ux + uy * uy) * R(a.inv_c2));
        const R rx = finite ? R(a.dt) * ux * ginv : R(0);
        const R ry = finite ? R(a.dt) * uy * ginv : R(0);

        // First straight piece, in the start triangle (Sec. II.D).
        const Piece<R> pc = trace_piece(g, l0, l1, l2, s0, s1, s2, r, rx, ry, -1);
        nseg += alive ? 1 : 0;
        if (alive && !finite) {
            atomicOr(a.counters + 2, 2ull);
            atomicMin(a.counters + 3, (unsigned long long)(a.pid ? a.pid[i] : i));
        }
        const bool leaving = alive && finite && !pc.done;
        if (alive && !leaving) finish_particle<R>(a, i, f, r, l0, l1, l2, finite, false, nlost);
        const int nbf = pick(pc.ks < 0 ? 0 : pc.ks, nb.x, nb.y, nb.z);
        const int kk = (nb.w >> (2 * (pc.ks < 0 ? 0 : pc.ks))) & 3;

        // Queue the particles leaving their triangle (one LDS atomic per
        // wavefront); overflow is finished in place.
        const unsigned long long lm = __ballot(leaving);
        if (lm) {
            int base = 0;
            if (lane == 0) base = atomicAdd(&s_qn, __popcll(lm));
            base = __shfl(base, 0, 64);
            const int slot = base + __popcll(lm & ((1ull << lane) - 1ull));
            if (leaving) {
                if (slot < kQueue) {
                    s_q.idx[slot] = i;
                    s_q.fk[slot] = nbf < 0 ? kLost : (uint32_t(nbf) | (uint32_t(kk) << 30));
                    s_q.ts[slot] = pc.ts;
                    s_q.la[slot] = pc.la;
                    s_q.rx[slot] = rx;
                    s_q.ry[slot] = ry;
                } else {
                    bool capped = false;
                    uint32_t fe = f;
                    int re = r;
                    R m0 = R(0), m1 = R(0), m2 = R(0);
                    const bool ok = continue_track(m, dep, q, a.cap, fe, re, nbf, kk, pc.la, pc.ts,
                                                   m0, m1, m2, rx, ry, nseg, capped);
                    finish_particle<R>(a, i, fe, re, m0, m1, m2, ok, capped, nlost);
                }
            }
        }

        // Wavefront segmented sum of the first-piece currents over runs of
        // equal start triangle, then one LDS add per edge and run.
        const int f0 = alive ? int(f) : -1;
        double c0 = alive ? pc.w0 : 0.0, c1 = alive ? pc.w1 : 0.0, c2 = alive ? pc.w2 : 0.0;
        const int kprev = __shfl_up(f0, 1, 64);
        const bool head = lane == 0 || kprev != f0;
        const unsigned long long hm = __ballot(head);
        const unsigned long long below = hm & ((2ull << lane) - 1ull);
        const int seg_start = 63 - __clzll(below);
        wave_segmented_sum(c0, c1, c2, lane, seg_start);
        const bool tail = lane == 63 || ((hm >> (lane + 1)) & 1ull);
        if (tail && f0 >= 0) {
            dep.add(te.x, ((te.w & 1) ? -q : q) * c0);
            dep.add(te.y, ((te.w & 2) ? -q : q) * c1);
            dep.add(te.z, ((te.w & 4) ? -q : q) * c2);
        }
    }

    // Phase 2: finish the queued particles, all lanes busy.
    __syncthreads();
    const int nq = s_qn < kQueue ? s_qn : kQueue;
    for (int t = threadIdx.x; t < nq; t += kBlock) {
        const uint32_t i = s_q.idx[t];
        const uint32_t fk = s_q.fk[t];
        const int nbf = fk == kLost ? -1 : int(fk & kTriMask);
        const int kk = int(fk >> 30);
        uint32_t f = 0;
        int r = 0;
        R l0 = R(0), l1 = R(0), l2 = R(0);
        bool capped = false;
        const bool ok = continue_track(m, dep, q, a.cap, f, r, nbf, kk, s_q.la[t], s_q.ts[t], l0, l1,
                                       l2, s_q.rx[t], s_q.ry[t], nseg, capped);
        finish_particle<R>(a, i, f, r, l0, l1, l2, ok, capped, nlost);
    }

    // Flush the block's currents: one global FP64 atomic per touched edge
    // of the window (a slot is non-zero only if an edge in range was added).
    __syncthreads();
    for (int t = threadIdx.x; t < kWin; t += kBlock) {
        const double v = s_acc[t];
        if (v != 0.0) atomic_add_f64(a.cur + wbase + uint32_t(t), v);
    }

    // Counters: per-block running sums in the block's own slot (launches on
    // one stream are ordered, so no atomics are needed).
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        nseg += __shfl_down(nseg, off, 64);
        nlost += __shfl_down(nlost, off, 64);
    }
    if (lane == 0) {
        red[0][threadIdx.x >> 6] = nseg;
        red[1][threadIdx.x >> 6] = nlost;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s0 = 0, s1 = 0;
#pragma unroll
        for (int wv = 0; wv < kBlock / 64; ++wv) {
            s0 += red[0][wv];
            s1 += red[1][wv];
        }
        a.block_counts[2 * tile] += s0;
        a.block_counts[2 * tile + 1] += s1;
    }
    __syncthreads();
}

// Occupancy target of the single-run particle kernel: 5 wavefronts per
// SIMD in FP32 (fits without spilling), 4 in FP64.  The batched kernel
// (more live state per tile) targets 4.
template <typename R>
constexpr int kWavesPerEU = sizeof(R) == 4 ? 5 : 4;

template <int P, typename R>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kWavesPerEU<R>)))
void k_particle_step(MeshView m, StepArgs a)
{
    __shared__ TileShared<R> sh;
    particle_tile<P, R>(m, a, uint32_t(xcd_tile(blockIdx.x, gridDim.x)), sh);
}

// Batched particle stage: many (run, species) segments in one persistent
// launch; blocks walk the flattened tile list.
template <int P, typename R>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
void k_particle_batched(const SegDesc *__restrict__ segs, const uint32_t *__restrict__ tile_prefix,
                        int nseg, uint32_t total_tiles)
{
    __shared__ TileShared<R> sh;
    for (uint32_t g = blockIdx.x; g < total_tiles; g += gridDim.x) {
        int lo = 0, hi = nseg - 1;  // last segment with tile_prefix[s] <= g
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tile_prefix[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        const SegDesc &sd = segs[lo];
        particle_tile<P, R>(sd.m, sd.a, g - tile_prefix[lo], sh);
    }
}

// ---------------------------------------------------------------------
// Faraday half step and per-triangle gather record.
// ---------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void faraday_tri(int f, const int4 *__restrict__ tri_edge,
                                            const double *__restrict__ e,
                                            const double *__restrict__ e_ext, double e_scale,
                                            double *__restrict__ b,
                                            const double *__restrict__ damp_b,
                                            double *__restrict__ h,
                                            const double *__restrict__ inv_mu_area,
                                            const double *__restrict__ inv_2area,
                                            const double *__restrict__ bz_ext,
                                            const double *__restrict__ grad, R *__restrict__ rec,
                                            double dt)
{
    const int4 te = tri_edge[f];
    const double e0 = e[te.x], e1 = e[te.y], e2 = e[te.z];
    const double s0 = (te.w & 1) ? -e0 : e0;
    const double s1 = (te.w & 2) ? -e1 : e1;
    const double s2 = (te.w & 4) ? -e2 : e2;
    const double bo = b[f];
    double bn = bo - dt * ((s0 + s1) + s2);
    if (damp_b) bn = bn * damp_b[f];  // matched magnetic loss of the absorbing layer
    b[f] = bn;
    h[f] = bn * inv_mu_area[f];
    double bz = (bn + bo) * inv_2area[f];
    if (bz_ext) bz += bz_ext[f];
    double t0 = s0, t1 = s1, t2 = s2;
    if (e_ext) {
        // applied field scaled (rounded product, not fused into the sum)
        const double x0 = __dmul_rn(e_scale, e_ext[te.x]);
        const double x1 = __dmul_rn(e_scale, e_ext[te.y]);
        const double x2 = __dmul_rn(e_scale, e_ext[te.z]);
        t0 = (te.w & 1) ? -(e0 + x0) : (e0 + x0);
        t1 = (te.w & 2) ? -(e1 + x1) : (e1 + x1);
        t2 = (te.w & 4) ? -(e2 + x2) : (e2 + x2);
    }
    const double *g = grad + size_t(f) * 6;
    // E = sum_k s_k (l_a grad l_b - l_b grad l_a) = sum_n l_n V_n with
    // V_n = s_{n+2} grad l_{n+1} - s_{n+1} grad l_{n+2}.
    R *o = rec + size_t(f) * 8;
    o[0] = R(t2 * g[2] - t1 * g[4]);
    o[1] = R(t2 * g[3] - t1 * g[5]);
    o[2] = R(t0 * g[4] - t2 * g[0]);
    o[3] = R(t0 * g[5] - t2 * g[1]);
    o[4] = R(t1 * g[0] - t0 * g[2]);
    o[5] = R(t1 * g[1] - t0 * g[3]);
    o[6] = R(bz);
    o[7] = R(0);
}

template <typename R>
__global__ __launch_bounds__(256) void k_faraday(int nf, const int4 *__restrict__ tri_edge,
                                                 const double *__restrict__ e,
                                                 const double *__restrict__ e_ext, double e_scale,
                                                 double *__restrict__ b,
                                                 const double *__restrict__ damp_b,
                                                 double *__restrict__ h,
                                                 const double *__restrict__ inv_mu_area,
                                                 const double *__restrict__ inv_2area,
                                                 const double *__restrict__ bz_ext,
                                                 const double *__restrict__ grad,
                                                 R *__restrict__ rec, double dt)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < nf)
        faraday_tri<R>(f, tri_edge, e, e_ext, e_scale, b, damp_b, h, inv_mu_area, inv_2area, bz_ext,
                       grad, rec, dt);
}

// Run of a batched field-stage block: the last run whose block prefix is
// <= g (runs hold ceil(n/256) blocks each).
__device__ __forceinline__ int run_of(const uint32_t *__restrict__ prefix, int nrun, uint32_t g)
{
    int lo = 0, hi = nrun - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_faraday_batched(const FieldDesc *__restrict__ runs,
                                                         const uint32_t *__restrict__ prefix,
                                                         int nrun, uint32_t total_blocks)
{
    for (uint32_t g = blockIdx.x; g < total_blocks; g += gridDim.x) {
        const int r = run_of(prefix, nrun, g);
        const FieldDesc &d = runs[r];
        const int f = int(g - prefix[r]) * 256 + int(threadIdx.x);
        if (f >= d.nf) continue;
        if (d.rec_fp32)
            faraday_tri<float>(f, d.tri_edge, d.e, d.e_ext, d.e_scale, d.b, d.damp_b, d.h,
                             d.inv_mu_area, d.inv_2area, d.bz_ext, d.grad64,
                             static_cast<float *>(d.rec), d.dt);
        else
            faraday_tri<double>(f, d.tri_edge, d.e, d.e_ext, d.e_scale, d.b, d.damp_b, d.h,
                             d.inv_mu_area, d.inv_2area, d.bz_ext, d.grad64,
                             static_cast<double *>(d.rec), d.dt);
    }
}

// ---------------------------------------------------------------------
// Ampere half step on the primary state d (FP64).
// edge_face[e] = {f0, f1 (-1 on a wall), sign0, sign1}.
// ---------------------------------------------------------------------
__device__ __forceinline__ void ampere_edge(int ed, const int4 *__restrict__ edge_face,
                                            const double *__restrict__ h, double *__restrict__ cur,
                                            double *__restrict__ cur_last, double *__restrict__ d,
                                            const double *__restrict__ damp, double dt)
{
    const double ie = cur[ed];
    cur_last[ed] = ie;
    cur[ed] = 0.0;
    const int4 ef = edge_face[ed];
    if (ef.y < 0) return;  // wall edge: not a free DoF, d stays 0
    const double curl = double(ef.z) * h[ef.x] + double(ef.w) * h[ef.y];
    double dn = d[ed] + dt * (curl - ie);
    if (damp) dn *= damp[ed];
    d[ed] = dn;
}

__global__ __launch_bounds__(256) void k_ampere(int ne, const int4 *__restrict__ edge_face,
                                                const double *__restrict__ h,
                                                double *__restrict__ cur,
                                                double *__restrict__ cur_last,
                                                double *__restrict__ d,
                                                const double *__restrict__ damp, double dt)
{
    const int ed = blockIdx.x * blockDim.x + threadIdx.x;
    if (ed < ne) ampere_edge(ed, edge_face, h, cur, cur_last, d, damp, dt);
}

// e = M~ d, M~ in SELL-64 (slices of 64 rows, column-major inside a slice).
__device__ __forceinline__ void spmv_row(int row, const int32_t *__restrict__ slice_ptr,
                                         const int32_t *__restrict__ slice_w,
                                         const int32_t *__restrict__ col,
                                         const double *__restrict__ val,
                                         const double *__restrict__ d, double *__restrict__ e)
{
    const int sl = row / kSlice, ln = row % kSlice;
    const int base = slice_ptr[sl], w = slice_w[sl];
    double acc = 0.0;
    for (int j = 0; j < w; ++j) {
        const int q = base + j * kSlice + ln;
        acc += val[q] * d[col[q]];
    }
    e[row] = acc;
}

__global__ __launch_bounds__(256) void k_spmv(int ne, const int32_t *__restrict__ slice_ptr,
                                              const int32_t *__restrict__ slice_w,
                                              const int32_t *__restrict__ col,
                                              const double *__restrict__ val,
                                              const double *__restrict__ d,
                                              double *__restrict__ e)
{
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row < ne) spmv_row(row, slice_ptr, slice_w, col, val, d, e);
}

__global__ __launch_bounds__(256) void k_ampere_batched(const FieldDesc *__restrict__ runs,
                                                        const uint32_t *__restrict__ prefix,
                                                        int nrun, uint32_t total_blocks)
{
    for (uint32_t g = blockIdx.x; g < total_blocks; g += gridDim.x) {
        const int r = run_of(prefix, nrun, g);
        const FieldDesc &d = runs[r];
        const int ed = int(g - prefix[r]) * 256 + int(threadIdx.x);
        if (ed < d.ne) ampere_edge(ed, d.edge_face, d.h, d.cur, d.cur_last, d.d, d.damp, d.dt);
    }
}

__global__ __launch_bounds__(256) void k_spmv_batched(const FieldDesc *__restrict__ runs,
                                                      const uint32_t *__restrict__ prefix,
                                                      int nrun, uint32_t total_blocks)
{
    for (uint32_t g = blockIdx.x; g < total_blocks; g += gridDim.x) {
        const int r = run_of(prefix, nrun, g);
        const FieldDesc &d = runs[r];
        const int row = int(g - prefix[r]) * 256 + int(threadIdx.x);
        if (row < d.ne) spmv_row(row, d.sl_ptr, d.sl_w, d.sl_col, d.sl_val, d.d, d.e_out);
    }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *__restrict__ p, uint32_t v, int64_t n)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------
// Counting sort by triangle, aggregated per block.  Between sorts the
// particles move to nearby triangles, so a block of kSortB consecutive
// particles covers a short triangle range: the block counts in an LDS
// histogram over kSortBins triangles anchored kSortBack before the home
// triangle of its first tile (from the previous sort) and adds one global
// count per touched triangle; triangles outside the window are counted
// directly.  The scatter ranks particles in the same LDS bins, reserves one
// global range per touched triangle and writes the block's particles out in
// triangle order (consecutive threads, consecutive destinations).
// ---------------------------------------------------------------------
constexpr int kSortPer = 8;
constexpr int kSortB = 256 * kSortPer;
constexpr int kSortBins = 1024;
constexpr uint32_t kSortBack = 256;

__device__ __forceinline__ uint32_t sort_window(const SortArgs &a, int64_t blk)
{
    if (!a.tile_home) return 0u;
    const uint32_t h = a.tile_home[(blk * kSortB) / (kPPT * kBlock)];
    return h > kSortBack ? h - kSortBack : 0u;
}

__global__ __launch_bounds__(256) void k_sort_hist(SortArgs a)
{
    __shared__ int32_t h[kSortBins];
    for (int t = threadIdx.x; t < kSortBins; t += 256) h[t] = 0;
    const uint32_t wb = sort_window(a, blockIdx.x);
    __syncthreads();
    const int64_t b0 = int64_t(blockIdx.x) * kSortB;
#pragma unroll
    for (int j = 0; j < kSortPer; ++j) {
        const int64_t i = b0 + j * 256 + int(threadIdx.x);
        const uint32_t k = i < a.n ? a.key_in[i] : kLost;
        if (k == kLost) continue;
        const uint32_t f = k & kTriMask, bin = f - wb;
        if (bin < uint32_t(kSortBins)) atomicAdd(&h[bin], 1);
        else atomicAdd(a.counts + f, 1);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kSortBins; t += 256)
        if (h[t]) atomicAdd(a.counts + wb + uint32_t(t), h[t]);
}

// Exclusive scan of counts[0..n) into offsets[0..n], three passes.
__global__ __launch_bounds__(1024) void k_scan_blocks(int n, const int32_t *__restrict__ in,
                                                      int32_t *__restrict__ out,
                                                      int32_t *__restrict__ block_sums)
{
    __shared__ int32_t s[1024];
    const int i = blockIdx.x * 1024 + threadIdx.x;
    const int v = i < n ? in[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n) out[i] = s[threadIdx.x] - v;
    if (threadIdx.x == 1023) block_sums[blockIdx.x] = s[1023];
}

__global__ __launch_bounds__(1024) void k_scan_sums(int nb, int32_t *__restrict__ block_sums)
{
    // single block, nb <= 1024 * per_thread
    __shared__ int32_t s[1024];
    const int per = (nb + 1023) / 1024;
    int local = 0;
    for (int j = 0; j < per; ++j) {
        const int idx = threadIdx.x * per + j;
        if (idx < nb) local += block_sums[idx];
    }
    s[threadIdx.x] = local;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    int run = s[threadIdx.x] - local;
    for (int j = 0; j < per; ++j) {
        const int idx = threadIdx.x * per + j;
        if (idx < nb) {
            const int v = block_sums[idx];
            block_sums[idx] = run;
            run += v;
        }
    }
    if (threadIdx.x == 1023) block_sums[nb] = s[1023];
}

__global__ __launch_bounds__(1024) void k_scan_add(int n, int32_t *__restrict__ out,
                                                   const int32_t *__restrict__ block_sums,
                                                   int nb)
{
    const int i = blockIdx.x * 1024 + threadIdx.x;
    if (i < n) out[i] += block_sums[blockIdx.x];
    if (i == 0) out[n] = block_sums[nb];
}

template <typename E>
__global__ __launch_bounds__(256) void k_sort_scatter(SortArgs a)
{
    __shared__ int32_t cnt[kSortBins];   // local count, then global base per bin
    __shared__ int32_t loc[kSortBins];   // local exclusive offset per bin
    __shared__ int32_t wsum[4];
    __shared__ int32_t n_out;            // particles outside the window
    __shared__ uint16_t s_src[kSortB];   // local slot -> block-local input index
    __shared__ int32_t s_dst[kSortB];    // local slot -> destination
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int t = tid; t < kSortBins; t += 256) cnt[t] = 0;
    if (tid == 0) n_out = 0;
    const uint32_t wb = sort_window(a, blockIdx.x);
    __syncthreads();
    const int64_t b0 = int64_t(blockIdx.x) * kSortB;
    // ranks within the block's bins (outside the window: a direct global slot)
    int32_t bin[kSortPer], rank[kSortPer];
#pragma unroll
    for (int j = 0; j < kSortPer; ++j) {
        const int64_t i = b0 + j * 256 + tid;
        const uint32_t k = i < a.n ? a.key_in[i] : kLost;
        bin[j] = -1;
        rank[j] = -1;
        if (k == kLost) continue;
        const uint32_t f = k & kTriMask, b = f - wb;
        if (b < uint32_t(kSortBins)) {
            bin[j] = int32_t(b);
            rank[j] = atomicAdd(&cnt[b], 1);
        } else {
            bin[j] = -2;
            rank[j] = atomicAdd(&n_out, 1);
            s_dst[kSortB - 1 - rank[j]] = a.offsets[f] + atomicAdd(a.counts + f, 1);
            s_src[kSortB - 1 - rank[j]] = uint16_t(j * 256 + tid);
        }
    }
    __syncthreads();
    // exclusive scan of the bin counts (4 per thread), then one global
    // reservation per touched triangle
    int32_t c4[4], run = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        c4[q] = cnt[4 * tid + q];
        run += c4[q];
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
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int b = 4 * tid + q;
        loc[b] = before;
        before += c4[q];
        cnt[b] = c4[q] ? a.offsets[wb + uint32_t(b)] + atomicAdd(a.counts + wb + uint32_t(b), c4[q])
                       : 0;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortPer; ++j) {
        if (bin[j] < 0) continue;
        const int slot = loc[bin[j]] + rank[j];
        s_src[slot] = uint16_t(j * 256 + tid);
        s_dst[slot] = cnt[bin[j]] + rank[j];
    }
    __syncthreads();
    // copy out in slot order: in-window slots [0, n_in), outside ones at the top
    const int n_in = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    const int nout = n_out;
    for (int s = tid; s < kSortB; s += 256) {
        if (s >= n_in && s < kSortB - nout) continue;
        const int64_t src = b0 + s_src[s];
        const int64_t dst = s_dst[s];
        a.key_out[dst] = a.key_in[src];
        reinterpret_cast<E *>(a.lam_out)[dst] = reinterpret_cast<const E *>(a.lam_in)[src];
        reinterpret_cast<E *>(a.u_out)[dst] = reinterpret_cast<const E *>(a.u_in)[src];
        a.pid_out[dst] = a.pid_in[src];
    }
}

// Home triangle of every tile of the sorted segment (its first particle).
__global__ __launch_bounds__(256) void k_tile_home(int64_t n, const uint32_t *__restrict__ key,
                                                   uint32_t *__restrict__ home, int64_t tiles)
{
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= tiles) return;
    const int64_t i = t * int64_t(kPPT * kBlock);
    const uint32_t k = i < n ? key[i] : kLost;
    home[t] = k == kLost ? 0u : (k & kTriMask);
}

// ---------------------------------------------------------------------
// Field probes: E = sum_k s_k e_k (l_a grad l_b - l_b grad l_a) (Sec. II.B)
// at fixed points, accumulated over a window of steps; at the end of a
// window the average is written out and the sum restarts.
// ---------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_probe(int n, const int32_t *__restrict__ tri,
                                               const double *__restrict__ lam,
                                               const int4 *__restrict__ tri_edge,
                                               const double *__restrict__ grad,
                                               const double *__restrict__ e,
                                               double *__restrict__ acc, double *__restrict__ out,
                                               double inv_window)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int f = tri[i];
    const double l1 = lam[2 * i], l2 = lam[2 * i + 1];
    const double l0 = (1.0 - l1) - l2;
    const int4 te = tri_edge[f];
    const double *g = grad + size_t(f) * 6;
    const double s0 = (te.w & 1) ? -e[te.x] : e[te.x];
    const double s1 = (te.w & 2) ? -e[te.y] : e[te.y];
    const double s2 = (te.w & 4) ? -e[te.z] : e[te.z];
    // local edge k joins nodes a = k+1, b = k+2
    const double ex = s0 * (l1 * g[4] - l2 * g[2]) + s1 * (l2 * g[0] - l0 * g[4]) +
                      s2 * (l0 * g[2] - l1 * g[0]);
    const double ey = s0 * (l1 * g[5] - l2 * g[3]) + s1 * (l2 * g[1] - l0 * g[5]) +
                      s2 * (l0 * g[3] - l1 * g[1]);
    double ax = acc[2 * i] + ex, ay = acc[2 * i + 1] + ey;
    if (out) {
        out[2 * i] = ax * inv_window;
        out[2 * i + 1] = ay * inv_window;
        ax = 0.0;
        ay = 0.0;
    }
    acc[2 * i] = ax;
    acc[2 * i + 1] = ay;
}

// ---------------------------------------------------------------------
// Diagnostics.
// ---------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_charge(int64_t n, const uint32_t *__restrict__ key,
                                                const void *__restrict__ lamv,
                                                const int4 *__restrict__ tri_node, double qw,
                                                double *__restrict__ q)
{
    using R2 = typename Vec2<R>::type;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = key[i];
    if (k == kLost) return;
    const R2 pr = reinterpret_cast<const R2 *>(lamv)[i];
    const int f = int(k & kTriMask), r = int(k >> 30);
    Tri3<double> L;
    L.set(next3(r), double(pr.x));
    L.set(prev3(r), double(pr.y));
    L.set(r, (1.0 - double(pr.x)) - double(pr.y));
    const int4 tn = tri_node[f];
    atomic_add_f64(q + tn.x, qw * L.v0);
    atomic_add_f64(q + tn.y, qw * L.v1);
    atomic_add_f64(q + tn.z, qw * L.v2);
}

__global__ __launch_bounds__(256) void k_divd(int ne, const int2 *__restrict__ en,
                                              const double *__restrict__ d,
                                              double *__restrict__ out)
{
    const int ed = blockIdx.x * blockDim.x + threadIdx.x;
    if (ed >= ne) return;
    const int2 p = en[ed];
    atomic_add_f64(out + p.x, d[ed]);
    atomic_add_f64(out + p.y, -d[ed]);
}

template <typename R>
__global__ __launch_bounds__(256) void k_kinetic(int64_t n, const uint32_t *__restrict__ key,
                                                 const void *__restrict__ uv, double inv_c2,
                                                 double *__restrict__ partial, int n_partial)
{
    using R2 = typename Vec2<R>::type;
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        if (key[i] == kLost) continue;
        const R2 u = reinterpret_cast<const R2 *>(uv)[i];
        const double u2 = (double(u.x) * double(u.x) + double(u.y) * double(u.y)) * inv_c2;
        // gamma - 1 = u2 / (sqrt(1 + u2) + 1), without cancellation
        acc += u2 / (sqrt(1.0 + u2) + 1.0);
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0 && blockIdx.x < n_partial) partial[blockIdx.x] = s[0];
}

inline unsigned grid_for(int64_t n, int block) { return unsigned((n + block - 1) / block); }

}  // namespace

hipError_t launch_faraday(hipStream_t s, int nf, const int4 *tri_edge, const double *e,
                          const double *e_ext, double e_scale, double *b, const double *damp_b,
                          double *h,
                          const double *inv_mu_area, const double *inv_2area,
                          const double *bz_ext, const double *grad64, void *rec, bool rec_fp32,
                          double dt)
{
    if (nf <= 0) return hipSuccess;
    if (rec_fp32)
        FETD_LAUNCH(k_faraday<float>, dim3(grid_for(nf, 256)), dim3(256), 0, s, nf,
                           tri_edge, e, e_ext, e_scale, b, damp_b, h, inv_mu_area, inv_2area,
                           bz_ext, grad64, static_cast<float *>(rec), dt);
    else
        FETD_LAUNCH(k_faraday<double>, dim3(grid_for(nf, 256)), dim3(256), 0, s, nf,
                           tri_edge, e, e_ext, e_scale, b, damp_b, h, inv_mu_area, inv_2area,
                           bz_ext, grad64, static_cast<double *>(rec), dt);
    return hipGetLastError();
}

template <int P>
static void launch_particles_p(hipStream_t s, const MeshView &m, const StepArgs &a, bool fp32)
{
    const unsigned grid = grid_for(a.n, int64_t(kBlock) * kPPT);
    if (fp32)
        FETD_LAUNCH((k_particle_step<P, float>), dim3(grid), dim3(kBlock), 0, s, m, a);
    else
        FETD_LAUNCH((k_particle_step<P, double>), dim3(grid), dim3(kBlock), 0, s, m, a);
}

hipError_t launch_particles(hipStream_t s, const MeshView &m, const StepArgs &a, int pusher,
                            bool fp32)
{
    if (a.n <= 0) return hipSuccess;
    switch (pusher) {
    case 0: launch_particles_p<0>(s, m, a, fp32); break;
    case 1: launch_particles_p<1>(s, m, a, fp32); break;
    case 2: launch_particles_p<2>(s, m, a, fp32); break;
    case 3: launch_particles_p<3>(s, m, a, fp32); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ampere(hipStream_t s, int ne, const int4 *edge_face, const double *h,
                         double *cur, double *cur_last, double *d, const double *damp, double dt)
{
    if (ne <= 0) return hipSuccess;
    FETD_LAUNCH(k_ampere, dim3(grid_for(ne, 256)), dim3(256), 0, s, ne, edge_face, h, cur,
                       cur_last, d, damp, dt);
    return hipGetLastError();
}

hipError_t launch_spmv(hipStream_t s, int ne, const int32_t *slice_ptr, const int32_t *slice_w,
                       const int32_t *col, const double *val, const double *d, double *e)
{
    if (ne <= 0) return hipSuccess;
    FETD_LAUNCH(k_spmv, dim3(grid_for(ne, 256)), dim3(256), 0, s, ne, slice_ptr, slice_w,
                       col, val, d, e);
    return hipGetLastError();
}

hipError_t launch_probe(hipStream_t s, int n, const int32_t *tri, const double *lam,
                        const int4 *tri_edge, const double *grad64, const double *e, double *acc,
                        double *out, double inv_window)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe, dim3(grid_for(n, 256)), dim3(256), 0, s, n, tri, lam, tri_edge,
                       grad64, e, acc, out, inv_window);
    return hipGetLastError();
}

hipError_t launch_fill_u32(hipStream_t s, uint32_t *p, uint32_t v, int64_t n)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_sort(hipStream_t s, const SortArgs &a)
{
    // fill kernels rather than memsets, so the sort can sit in a captured graph
    hipError_t err = launch_fill_u32(s, reinterpret_cast<uint32_t *>(a.counts), 0u, a.nf + 1);
    if (err != hipSuccess) return err;
    err = launch_fill_u32(s, a.key_out, kLost, a.n);
    if (err != hipSuccess) return err;
    if (a.n > 0)
        hipLaunchKernelGGL(k_sort_hist, dim3(grid_for(a.n, kSortB)), dim3(256), 0, s, a);
    const int nb = int((a.nf + 1023) / 1024);
    hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(1024), 0, s, a.nf, a.counts, a.offsets,
                       a.block_sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, nb, a.block_sums);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(1024), 0, s, a.nf, a.offsets, a.block_sums, nb);
    err = launch_fill_u32(s, reinterpret_cast<uint32_t *>(a.counts), 0u, a.nf + 1);
    if (err != hipSuccess) return err;
    if (a.n > 0) {
        if (a.elem_bytes == 8)
            hipLaunchKernelGGL(k_sort_scatter<float2>, dim3(grid_for(a.n, kSortB)), dim3(256), 0,
                               s, a);
        else
            hipLaunchKernelGGL(k_sort_scatter<double2>, dim3(grid_for(a.n, kSortB)), dim3(256), 0,
                               s, a);
    }
    if (a.tile_home && a.n > 0) {
        const int64_t tiles = (a.n + int64_t(kPPT * kBlock) - 1) / int64_t(kPPT * kBlock);
        hipLaunchKernelGGL(k_tile_home, dim3(grid_for(tiles, 256)), dim3(256), 0, s, a.n,
                           a.key_out, a.tile_home, tiles);
    }
    return hipGetLastError();
}

static unsigned persistent_grid(uint32_t total, unsigned per_cu)
{
    const uint32_t cap = 256u * per_cu;
    return total < cap ? (total > 0 ? total : 1u) : cap;
}

hipError_t launch_faraday_batched(hipStream_t s, const FieldDesc *d, const uint32_t *prefix,
                                  int nrun, uint32_t total_blocks)
{
    if (total_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_faraday_batched, dim3(persistent_grid(total_blocks, 8)), dim3(256), 0, s,
                       d, prefix, nrun, total_blocks);
    return hipGetLastError();
}

hipError_t launch_ampere_batched(hipStream_t s, const FieldDesc *d, const uint32_t *prefix,
                                 int nrun, uint32_t total_blocks)
{
    if (total_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ampere_batched, dim3(persistent_grid(total_blocks, 8)), dim3(256), 0, s,
                       d, prefix, nrun, total_blocks);
    return hipGetLastError();
}

hipError_t launch_spmv_batched(hipStream_t s, const FieldDesc *d, const uint32_t *prefix,
                               int nrun, uint32_t total_blocks)
{
    if (total_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_spmv_batched, dim3(persistent_grid(total_blocks, 8)), dim3(256), 0, s,
                       d, prefix, nrun, total_blocks);
    return hipGetLastError();
}

// Blocks of a kernel resident per CU (HIP's occupancy calculator), so a
// persistent launch holds no block that would wait for others to finish
// their whole tile lists before it starts.
static unsigned resident_per_cu(const void *kernel, unsigned fallback)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kBlock, 0) != hipSuccess ||
        nb < 1)
        return fallback;
    return unsigned(nb);
}

template <int P>
static void launch_particles_batched_p(hipStream_t s, const SegDesc *segs, const uint32_t *prefix,
                                       int nseg, uint32_t total, bool fp32)
{
    if (fp32) {
        static const unsigned per_cu = resident_per_cu(
            reinterpret_cast<const void *>(&k_particle_batched<P, float>), 4);
        hipLaunchKernelGGL((k_particle_batched<P, float>), dim3(persistent_grid(total, per_cu)),
                           dim3(kBlock), 0, s, segs, prefix, nseg, total);
    } else {
        static const unsigned per_cu = resident_per_cu(
            reinterpret_cast<const void *>(&k_particle_batched<P, double>), 4);
        hipLaunchKernelGGL((k_particle_batched<P, double>), dim3(persistent_grid(total, per_cu)),
                           dim3(kBlock), 0, s, segs, prefix, nseg, total);
    }
}

hipError_t launch_particles_batched(hipStream_t s, const SegDesc *segs, const uint32_t *prefix,
                                    int nseg, uint32_t total_tiles, int pusher, bool fp32)
{
    if (total_tiles == 0) return hipSuccess;
    switch (pusher) {
    case 0: launch_particles_batched_p<0>(s, segs, prefix, nseg, total_tiles, fp32); break;
    case 1: launch_particles_batched_p<1>(s, segs, prefix, nseg, total_tiles, fp32); break;
    case 2: launch_particles_batched_p<2>(s, segs, prefix, nseg, total_tiles, fp32); break;
    case 3: launch_particles_batched_p<3>(s, segs, prefix, nseg, total_tiles, fp32); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_charge(hipStream_t s, int64_t n, const uint32_t *key, const void *lam,
                         bool fp32, const int4 *tri_node, double qw, double *q)
{
    if (n <= 0) return hipSuccess;
    if (fp32)
        hipLaunchKernelGGL(k_charge<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, n, key, lam,
                           tri_node, qw, q);
    else
        hipLaunchKernelGGL(k_charge<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, n, key, lam,
                           tri_node, qw, q);
    return hipGetLastError();
}

hipError_t launch_divd(hipStream_t s, int ne, const int2 *edge_nodes, const double *d,
                       double *out)
{
    if (ne <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_divd, dim3(grid_for(ne, 256)), dim3(256), 0, s, ne, edge_nodes, d, out);
    return hipGetLastError();
}

hipError_t launch_kinetic(hipStream_t s, int64_t n, const uint32_t *key, const void *u, bool fp32,
                          double inv_c2, double *partial, int n_partial)
{
    if (n <= 0) return hipSuccess;
    if (fp32)
        hipLaunchKernelGGL(k_kinetic<float>, dim3(n_partial), dim3(256), 0, s, n, key, u, inv_c2,
                           partial, n_partial);
    else
        hipLaunchKernelGGL(k_kinetic<double>, dim3(n_partial), dim3(256), 0, s, n, key, u,
                           inv_c2, partial, n_partial);
    return hipGetLastError();
}

}  // namespace fetd
