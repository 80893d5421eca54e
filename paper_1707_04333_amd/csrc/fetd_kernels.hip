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
        const R g0 = sqrt(one + (ux * ux + uy * uy) * inv_c2);
        const R vx = ux / g0, vy = uy / g0;
        const R upx = ux + ex + vy * bz + ex;
        const R upy = uy + ey - vx * bz + ey;
        const R gp2 = one + (upx * upx + upy * upy) * inv_c2;
        const R bb = bz * bz;
        const R sig = gp2 - bb;
        const R gn = sqrt(R(0.5) * (sig + sqrt(sig * sig + R(4) * bb)));
        const R tz = bz / gn;
        const R s = one / (one + tz * tz);
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
        const R gh = sqrt(R(0.5) * (sig + sqrt(sig * sig + R(4) * bb)));
        tz = bz / gh;
    } else if constexpr (P == 1) {
        // Boris with the tan correction: t = (beta/|beta|) tan(|beta|/gbar).
        tz = tan(bz / sqrt(gm2));
    } else {
        tz = bz / sqrt(gm2);
    }
    const R sz = R(2) * tz / (one + tz * tz);
    const R qx = umx + umy * tz;   // u' = u- + u- x t
    const R qy = umy - umx * tz;
    ux = umx + qy * sz + ex;       // u+ = u- + u' x s, then the second half kick
    uy = umy - qx * sz + ey;
}

// ---------------------------------------------------------------------
// Block-local FP64 current accumulation: an open-addressing hash table in
// LDS keyed by edge id.  A block deposits every path piece of its
// particles here (LDS FP64 atomics) and flushes one global atomic per
// distinct edge at the end; the sorted order keeps the distinct edges of a
// block few.
// ---------------------------------------------------------------------
constexpr int kHashLog2 = 10;
constexpr int kHash = 1 << kHashLog2;
constexpr int kProbe = 32;

struct LdsCurrent {
    int *key;
    double *val;
    double *global;  // fallback when the table is congested

    __device__ __forceinline__ void add(int edge, double v) const
    {
        unsigned h = (unsigned(edge) * 2654435761u) >> (32 - kHashLog2);
#pragma nounroll
        for (int probe = 0; probe < kProbe; ++probe) {
            int k = __hip_atomic_load(key + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (k == -1) {
                int expected = -1;
                __hip_atomic_compare_exchange_strong(key + h, &expected, edge, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WORKGROUP);
                k = expected == -1 ? edge : expected;
            }
            if (k == edge) {
                __hip_atomic_fetch_add(val + h, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                return;
            }
            h = (h + 1) & (kHash - 1);
        }
        atomic_add_f64(global + edge, v);
    }
};

// ---------------------------------------------------------------------
// Fused particle stage: each block owns kPPT * kBlock consecutive
// (triangle-sorted) particles, one per thread per pass.
// ---------------------------------------------------------------------
template <int P, typename R>
__global__ __launch_bounds__(kBlock) void k_particle_step(MeshView m, StepArgs a)
{
    using R2 = typename Vec2<R>::type;
    __shared__ int s_key[kHash];
    __shared__ double s_val[kHash];
    __shared__ unsigned long long red[2][kBlock / 64];
    for (int t = threadIdx.x; t < kHash; t += kBlock) {
        s_key[t] = -1;
        s_val[t] = 0.0;
    }
    __syncthreads();
    const LdsCurrent dep{s_key, s_val, a.cur};
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x & 63;
    unsigned long long nseg = 0, nlost = 0;

    for (int pass = 0; pass < kPPT; ++pass) {
        const int64_t i = (tile * kPPT + pass) * kBlock + threadIdx.x;
        const bool in_range = i < a.n;
        uint32_t key = in_range ? a.key[i] : kLost;
        const bool alive = key != kLost;

        int f0 = -1;
        double c0 = 0.0, c1 = 0.0, c2 = 0.0;  // first path piece (cross terms)

        if (alive) {
            R2 *lamp = reinterpret_cast<R2 *>(a.lam);
            R2 *up = reinterpret_cast<R2 *>(a.u);
            R2 pr = lamp[i];
            R2 uu = up[i];
            int f = int(key & kTriMask);
            int r = int(key >> 30);
            f0 = f;

            Tri3<R> L;
            L.set(next3(r), pr.x);
            L.set(prev3(r), pr.y);
            L.set(r, (R(1) - pr.x) - pr.y);
            Tri3<double> Ls;  // FP64 start point of the current path piece
            Ls.set(next3(r), double(pr.x));
            Ls.set(prev3(r), double(pr.y));
            Ls.set(r, (1.0 - double(pr.x)) - double(pr.y));

            // Gather (Sec. II.B): E = sum_n l_n V_n from the triangle record.
            const R *rec = reinterpret_cast<const R *>(a.rec) + size_t(f) * 8;
            R ex = L.v0 * rec[0] + L.v1 * rec[2] + L.v2 * rec[4];
            R ey = L.v0 * rec[1] + L.v1 * rec[3] + L.v2 * rec[5];
            const R bzf = rec[6];
            if (a.has_affine) {
                R x, y;
                if constexpr (sizeof(R) == 4) {
                    const float *v = m.vxy32 + size_t(f) * 8;
                    x = L.v0 * v[0] + L.v1 * v[2] + L.v2 * v[4];
                    y = L.v0 * v[1] + L.v1 * v[3] + L.v2 * v[5];
                } else {
                    const double *v = m.vxy64 + size_t(f) * 6;
                    x = L.v0 * v[0] + L.v1 * v[2] + L.v2 * v[4];
                    y = L.v0 * v[1] + L.v1 * v[3] + L.v2 * v[5];
                }
                ex += R(a.aff[0]) + R(a.aff[2]) * x + R(a.aff[3]) * y;
                ey += R(a.aff[1]) + R(a.aff[4]) * x + R(a.aff[5]) * y;
            }

            // Push (Sec. II.C).
            const R alpha = R(a.alpha);
            R ux = uu.x, uy = uu.y;
            push2<P, R>(ux, uy, alpha * ex, alpha * ey, alpha * bzf, R(a.inv_c2));
            const bool finite = isfinite(ux) && isfinite(uy);

            // Move: dr = dt u / gamma (Sec. II.C eq. eq.motion.dis).
            const R ginv = R(1) / sqrt(R(1) + (ux * ux + uy * uy) * R(a.inv_c2));
            R rx = R(a.dt) * ux * ginv;
            R ry = R(a.dt) * uy * ginv;
            if (!finite) {
                rx = R(0);
                ry = R(0);
            }

            // Track across edges, depositing every straight piece (Sec. II.D).
            int entry = -1;
            bool lost = false, capped = false;
            for (int it = 0;; ++it) {
                if (it >= a.cap) {
                    capped = true;
                    break;
                }
                const R *g;
                if constexpr (sizeof(R) == 4) g = m.grad32 + size_t(f) * 8;
                else g = m.grad64 + size_t(f) * 6;
                Tri3<R> dL;
                dL.v0 = g[0] * rx + g[1] * ry;
                dL.v1 = g[2] * rx + g[3] * ry;
                dL.v2 = g[4] * rx + g[5] * ry;
                int ks = -1;
                R ts = R(0);
                if (entry != 0 && dL.v0 < R(0)) {
                    ks = 0;
                    ts = (L.v0 > R(0) ? L.v0 : R(0)) / (-dL.v0);
                }
                if (entry != 1 && dL.v1 < R(0)) {
                    const R tk = (L.v1 > R(0) ? L.v1 : R(0)) / (-dL.v1);
                    if (ks < 0 || tk < ts) {
                        ks = 1;
                        ts = tk;
                    }
                }
                if (entry != 2 && dL.v2 < R(0)) {
                    const R tk = (L.v2 > R(0) ? L.v2 : R(0)) / (-dL.v2);
                    if (ks < 0 || tk < ts) {
                        ks = 2;
                        ts = tk;
                    }
                }
                const bool done = ks < 0 || ts >= R(1);
                Tri3<double> Lf;
                R la = R(0);
                if (done) {
                    const int p = next3(r), q = prev3(r);
                    const R np = L.get(p) + dL.get(p);
                    const R nq = L.get(q) + dL.get(q);
                    L.set(p, np);
                    L.set(q, nq);
                    Lf.set(p, double(np));
                    Lf.set(q, double(nq));
                    Lf.set(r, (1.0 - double(np)) - double(nq));
                } else {
                    const int ia = next3(ks);
                    la = L.get(ia) + ts * dL.get(ia);
                    Lf.set(ks, 0.0);
                    Lf.set(ia, double(la));
                    Lf.set(prev3(ks), 1.0 - double(la));
                }
                // eq. I.assign for the three local edges (a, b) = (k+1, k+2).
                const double w0 = Ls.v1 * Lf.v2 - Lf.v1 * Ls.v2;
                const double w1 = Ls.v2 * Lf.v0 - Lf.v2 * Ls.v0;
                const double w2 = Ls.v0 * Lf.v1 - Lf.v0 * Ls.v1;
                ++nseg;
                if (it == 0) {
                    c0 = w0;
                    c1 = w1;
                    c2 = w2;
                } else {
                    const int4 te = m.tri_edge[f];
                    const double q = a.qdt;
                    dep.add(te.x, ((te.w & 1) ? -q : q) * w0);
                    dep.add(te.y, ((te.w & 2) ? -q : q) * w1);
                    dep.add(te.z, ((te.w & 4) ? -q : q) * w2);
                }
                if (done) break;
                const int4 nb = m.tri_nbr[f];
                const int nbf = ks == 0 ? nb.x : (ks == 1 ? nb.y : nb.z);
                if (nbf < 0) {
                    lost = true;
                    break;
                }
                // CCW neighbours traverse the shared edge in opposite
                // directions: node (ks+1) of f is node (kk+2) of the
                // neighbour and vice versa.
                const int kk = (nb.w >> (2 * ks)) & 3;
                const int a2 = next3(kk), b2 = prev3(kk);
                L.set(kk, R(0));
                L.set(b2, la);
                L.set(a2, R(1) - la);
                Ls.set(kk, 0.0);
                Ls.set(b2, double(la));
                Ls.set(a2, 1.0 - double(la));
                r = a2;
                f = nbf;
                entry = kk;
                const R sc = R(1) - ts;
                rx = rx * sc;
                ry = ry * sc;
            }
            if (capped || !finite) {
                atomicOr(a.counters + 2, capped ? 1ull : 2ull);
                atomicMin(a.counters + 3, (unsigned long long)(a.pid ? a.pid[i] : i));
                lost = true;
            }
            if (lost) {
                key = kLost;
                nlost += 1;
            } else {
                key = uint32_t(f) | (uint32_t(r) << 30);
                R2 np2;
                np2.x = L.get(next3(r));
                np2.y = L.get(prev3(r));
                lamp[i] = np2;
            }
            R2 un;
            un.x = ux;
            un.y = uy;
            up[i] = un;
            a.key[i] = key;
        }

        // Wavefront segmented sum of the first-piece currents over runs of
        // equal start triangle, then one LDS add per edge and run.
        const int kprev = __shfl_up(f0, 1, 64);
        const bool head = lane == 0 || kprev != f0;
        const unsigned long long hm = __ballot(head);
        const unsigned long long below = hm & ((2ull << lane) - 1ull);
        const int seg_start = 63 - __clzll(below);
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double o0 = __shfl_up(c0, off, 64);
            const double o1 = __shfl_up(c1, off, 64);
            const double o2 = __shfl_up(c2, off, 64);
            if (lane - off >= seg_start) {
                c0 += o0;
                c1 += o1;
                c2 += o2;
            }
        }
        const bool tail = lane == 63 || ((hm >> (lane + 1)) & 1ull);
        if (tail && f0 >= 0) {
            const int4 te = m.tri_edge[f0];
            const double q = a.qdt;
            dep.add(te.x, ((te.w & 1) ? -q : q) * c0);
            dep.add(te.y, ((te.w & 2) ? -q : q) * c1);
            dep.add(te.z, ((te.w & 4) ? -q : q) * c2);
        }
    }

    // Flush the block's currents: one global FP64 atomic per distinct edge.
    __syncthreads();
    for (int t = threadIdx.x; t < kHash; t += kBlock) {
        const int e = s_key[t];
        if (e >= 0) atomic_add_f64(a.cur + e, s_val[t]);
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
        a.block_counts[2 * blockIdx.x] += s0;
        a.block_counts[2 * blockIdx.x + 1] += s1;
    }
}

// ---------------------------------------------------------------------
// Faraday half step and per-triangle gather record.
// ---------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_faraday(int nf, const int4 *__restrict__ tri_edge,
                                                 const double *__restrict__ e,
                                                 const double *__restrict__ e_ext,
                                                 double *__restrict__ b, double *__restrict__ h,
                                                 const double *__restrict__ inv_mu_area,
                                                 const double *__restrict__ inv_2area,
                                                 const double *__restrict__ bz_ext,
                                                 const double *__restrict__ grad,
                                                 R *__restrict__ rec, double dt)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    const int4 te = tri_edge[f];
    const double e0 = e[te.x], e1 = e[te.y], e2 = e[te.z];
    const double s0 = (te.w & 1) ? -e0 : e0;
    const double s1 = (te.w & 2) ? -e1 : e1;
    const double s2 = (te.w & 4) ? -e2 : e2;
    const double bo = b[f];
    const double bn = bo - dt * ((s0 + s1) + s2);
    b[f] = bn;
    h[f] = bn * inv_mu_area[f];
    double bz = (bn + bo) * inv_2area[f];
    if (bz_ext) bz += bz_ext[f];
    double t0 = s0, t1 = s1, t2 = s2;
    if (e_ext) {
        const double x0 = e_ext[te.x], x1 = e_ext[te.y], x2 = e_ext[te.z];
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

// ---------------------------------------------------------------------
// Ampere half step on the primary state d (FP64).
// edge_face[e] = {f0, f1 (-1 on a wall), sign0, sign1}.
// ---------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ampere(int ne, const int4 *__restrict__ edge_face,
                                                const double *__restrict__ h,
                                                const double *__restrict__ cur,
                                                double *__restrict__ cur_next,
                                                double *__restrict__ d,
                                                const double *__restrict__ damp, double dt)
{
    const int ed = blockIdx.x * blockDim.x + threadIdx.x;
    if (ed >= ne) return;
    cur_next[ed] = 0.0;
    const int4 ef = edge_face[ed];
    if (ef.y < 0) return;  // wall edge: not a free DoF, d stays 0
    const double curl = double(ef.z) * h[ef.x] + double(ef.w) * h[ef.y];
    double dn = d[ed] + dt * (curl - cur[ed]);
    if (damp) dn *= damp[ed];
    d[ed] = dn;
}

// e = M~ d, M~ in SELL-64 (slices of 64 rows, column-major inside a slice).
__global__ __launch_bounds__(256) void k_spmv(int ne, const int32_t *__restrict__ slice_ptr,
                                              const int32_t *__restrict__ slice_w,
                                              const int32_t *__restrict__ col,
                                              const double *__restrict__ val,
                                              const double *__restrict__ d,
                                              double *__restrict__ e)
{
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= ne) return;
    const int sl = row / kSlice, ln = row % kSlice;
    const int base = slice_ptr[sl], w = slice_w[sl];
    double acc = 0.0;
    for (int j = 0; j < w; ++j) {
        const int q = base + j * kSlice + ln;
        acc += val[q] * d[col[q]];
    }
    e[row] = acc;
}

// ---------------------------------------------------------------------
// Counting sort by triangle.
// ---------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sort_hist(int64_t n, const uint32_t *__restrict__ key,
                                                   int32_t *__restrict__ counts)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint32_t k = i < n ? key[i] : kLost;
    const int lane = threadIdx.x & 63;
    const uint32_t kp = __shfl_up(k, 1, 64);
    const bool head = lane == 0 || kp != k;
    const unsigned long long hm = __ballot(head);
    const unsigned long long below = hm & ((2ull << lane) - 1ull);
    const int seg_start = 63 - __clzll(below);
    const bool tail = lane == 63 || ((hm >> (lane + 1)) & 1ull);
    if (tail && k != kLost) atomicAdd(counts + (k & kTriMask), lane - seg_start + 1);
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
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint32_t k = i < a.n ? a.key_in[i] : kLost;
    const int lane = threadIdx.x & 63;
    const uint32_t kp = __shfl_up(k, 1, 64);
    const bool head = lane == 0 || kp != k;
    const unsigned long long hm = __ballot(head);
    const unsigned long long below = hm & ((2ull << lane) - 1ull);
    const int seg_start = 63 - __clzll(below);
    const bool tail = lane == 63 || ((hm >> (lane + 1)) & 1ull);
    int base = 0;
    if (tail && k != kLost) {
        const int f = int(k & kTriMask);
        base = a.offsets[f] + atomicAdd(a.counts + f, lane - seg_start + 1);
    }
    // broadcast the run's base from its tail lane
    const unsigned long long tails = __ballot(tail);
    const unsigned long long at_or_above = tails & ~((1ull << lane) - 1ull);
    const int tail_lane = __ffsll((long long)at_or_above) - 1;
    base = __shfl(base, tail_lane, 64);
    if (k == kLost) return;
    const int64_t dst = int64_t(base) + (lane - seg_start);
    a.key_out[dst] = k;
    reinterpret_cast<E *>(a.lam_out)[dst] = reinterpret_cast<const E *>(a.lam_in)[i];
    reinterpret_cast<E *>(a.u_out)[dst] = reinterpret_cast<const E *>(a.u_in)[i];
    a.pid_out[dst] = a.pid_in[i];
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
                          const double *e_ext, double *b, double *h, const double *inv_mu_area,
                          const double *inv_2area, const double *bz_ext, const double *grad64,
                          void *rec, bool rec_fp32, double dt)
{
    if (nf <= 0) return hipSuccess;
    if (rec_fp32)
        hipLaunchKernelGGL(k_faraday<float>, dim3(grid_for(nf, 256)), dim3(256), 0, s, nf,
                           tri_edge, e, e_ext, b, h, inv_mu_area, inv_2area, bz_ext, grad64,
                           static_cast<float *>(rec), dt);
    else
        hipLaunchKernelGGL(k_faraday<double>, dim3(grid_for(nf, 256)), dim3(256), 0, s, nf,
                           tri_edge, e, e_ext, b, h, inv_mu_area, inv_2area, bz_ext, grad64,
                           static_cast<double *>(rec), dt);
    return hipGetLastError();
}

template <int P>
static void launch_particles_p(hipStream_t s, const MeshView &m, const StepArgs &a, bool fp32)
{
    const unsigned grid = grid_for(a.n, int64_t(kBlock) * kPPT);
    if (fp32)
        hipLaunchKernelGGL((k_particle_step<P, float>), dim3(grid), dim3(kBlock), 0, s, m, a);
    else
        hipLaunchKernelGGL((k_particle_step<P, double>), dim3(grid), dim3(kBlock), 0, s, m, a);
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
                         const double *cur, double *cur_next, double *d, const double *damp,
                         double dt)
{
    if (ne <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ampere, dim3(grid_for(ne, 256)), dim3(256), 0, s, ne, edge_face, h, cur,
                       cur_next, d, damp, dt);
    return hipGetLastError();
}

hipError_t launch_spmv(hipStream_t s, int ne, const int32_t *slice_ptr, const int32_t *slice_w,
                       const int32_t *col, const double *val, const double *d, double *e)
{
    if (ne <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_spmv, dim3(grid_for(ne, 256)), dim3(256), 0, s, ne, slice_ptr, slice_w,
                       col, val, d, e);
    return hipGetLastError();
}

hipError_t launch_sort(hipStream_t s, const SortArgs &a)
{
    hipError_t err = hipMemsetAsync(a.counts, 0, sizeof(int32_t) * size_t(a.nf + 1), s);
    if (err != hipSuccess) return err;
    if (a.n > 0)
        hipLaunchKernelGGL(k_sort_hist, dim3(grid_for(a.n, 256)), dim3(256), 0, s, a.n, a.key_in,
                           a.counts);
    const int nb = int((a.nf + 1023) / 1024);
    hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(1024), 0, s, a.nf, a.counts, a.offsets,
                       a.block_sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, nb, a.block_sums);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(1024), 0, s, a.nf, a.offsets, a.block_sums, nb);
    err = hipMemsetAsync(a.counts, 0, sizeof(int32_t) * size_t(a.nf + 1), s);
    if (err != hipSuccess) return err;
    if (a.n > 0) {
        if (a.elem_bytes == 8)
            hipLaunchKernelGGL(k_sort_scatter<float2>, dim3(grid_for(a.n, 256)), dim3(256), 0, s,
                               a);
        else
            hipLaunchKernelGGL(k_sort_scatter<double2>, dim3(grid_for(a.n, 256)), dim3(256), 0, s,
                               a);
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
