// HIP kernels (gfx950) of the field stages, the re-sort and the
// diagnostics of the charge-conserving relativistic FETD-PIC step.
//
// Method: arXiv:1707.04333 (Na, Moon, Omelchenko, Teixeira).  One step:
//   k_faraday        b^{n+1/2} = b^{n-1/2} - dt C e^n (Sec. II.A eq.
//                    semi.dis.curl.1), B^n = (B^{n+1/2} + B^{n-1/2})/2 (Sec.
//                    II.C) and the per-triangle field record of e^n;
//   k_particle_step  (fetd_particles.hip) gather, push, track, scatter;
//   k_ampere         d += dt (C^T [*mu^-1] b^{n+1/2} - i^{n+1/2})
//                    (Sec. II.A eq. semi.dis.curl.2 in the d = [*eps] e form);
//   k_spmv           e^{n+1} = M~ d^{n+1} with the sparse approximate inverse.
// Built with contraction off: each field update is the plain expression of
// its definition (b_new = b_old - dt ((s0 e0 + s1 e1) + s2 e2), h = b /
// (mu0 A), B^n = (b_new + b_old) / (2A), d + dt (curl - i)).
// The field state e, b, h and the values of M~ are FP64, or FP32 in the
// FP32-field mixed mode; d and the current are FP64 in every mode.
// Nothing here is a dense contraction: the kernels are bandwidth kernels.
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

__device__ __forceinline__ void atomic_add_f64(double *p, double v) { unsafeAtomicAdd(p, v); }

// Field arrays are FP64, or FP32 in the FP32-field mode.
template <typename FT>
__device__ __forceinline__ double fget(const void *p, int64_t i)
{
    return double(static_cast<const FT *>(p)[i]);
}
template <typename FT>
__device__ __forceinline__ void fset(void *p, int64_t i, double v)
{
    static_cast<FT *>(p)[i] = FT(v);
}

// ---------------------------------------------------------------------
// Faraday half step and per-triangle field record.
// ---------------------------------------------------------------------
template <typename FT>
__device__ __forceinline__ void faraday_tri(int f, const FieldDesc &d)
{
    const int4 te = d.tri_edge[f];
    const double e0 = fget<FT>(d.e, te.x), e1 = fget<FT>(d.e, te.y), e2 = fget<FT>(d.e, te.z);
    const double s0 = (te.w & 1) ? -e0 : e0;
    const double s1 = (te.w & 2) ? -e1 : e1;
    const double s2 = (te.w & 4) ? -e2 : e2;
    const double bo = fget<FT>(d.b, f);
    double bn = bo - d.dt * ((s0 + s1) + s2);
    if (d.damp_b) bn = bn * d.damp_b[f];  // matched magnetic loss of the absorbing layer
    fset<FT>(d.b, f, bn);
    const double bnr = fget<FT>(d.b, f);  // the stored (possibly FP32-rounded) value
    fset<FT>(d.h, f, bnr / d.mu_area[f]);
    double bz = (bnr + bo) / d.two_area[f];
    if (d.bz_ext) bz = bz + d.bz_ext[f];
    double t0 = s0, t1 = s1, t2 = s2;
    if (d.e_ext) {
        // applied field scaled (rounded product, then the sum with e)
        const double x0 = d.e_scale * d.e_ext[te.x];
        const double x1 = d.e_scale * d.e_ext[te.y];
        const double x2 = d.e_scale * d.e_ext[te.z];
        t0 = (te.w & 1) ? -(e0 + x0) : (e0 + x0);
        t1 = (te.w & 2) ? -(e1 + x1) : (e1 + x1);
        t2 = (te.w & 4) ? -(e2 + x2) : (e2 + x2);
    }
    if (d.rec_fp32) {
        // E = sum_k s_k (l_a grad l_b - l_b grad l_a) = sum_n l_n V_n with
        // V_n = s_{n+2} grad l_{n+1} - s_{n+1} grad l_{n+2}.
        const double *g = d.grad64 + size_t(f) * 6;
        float4 *o = static_cast<float4 *>(d.rec) + size_t(f) * 2;
        o[0] = make_float4(float(t2 * g[2] - t1 * g[4]), float(t2 * g[3] - t1 * g[5]),
                           float(t0 * g[4] - t2 * g[0]), float(t0 * g[5] - t2 * g[1]));
        o[1] = make_float4(float(t1 * g[0] - t0 * g[2]), float(t1 * g[1] - t0 * g[3]), float(bz),
                           0.f);
    } else {
        // the signed edge DoFs and B_z^n, gathered edge by edge
        double2 *o = static_cast<double2 *>(d.rec) + size_t(f) * 2;
        o[0] = make_double2(t0, t1);
        o[1] = make_double2(t2, bz);
    }
}

template <typename FT>
__global__ __launch_bounds__(256) void k_faraday(FieldDesc d)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < d.nf) faraday_tri<FT>(f, d);
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
        if (d.field32) faraday_tri<float>(f, d);
        else faraday_tri<double>(f, d);
    }
}

// ---------------------------------------------------------------------
// Ampere half step on the primary state d (FP64).
// edge_face[e] = {f0, f1 (-1 on a wall), sign0, sign1}.  In the
// deterministic mode the step's current is taken from the fixed-point
// limbs (and the limbs are cleared).
// ---------------------------------------------------------------------
__device__ __forceinline__ double fx_take(unsigned long long *p, double unscale)
{
    long long l0 = (long long)p[0], l1 = (long long)p[1], l2 = (long long)p[2];
    p[0] = 0ull;
    p[1] = 0ull;
    p[2] = 0ull;
    // carry: value = l0 + l1 2^32 + l2 2^64 with l0, l1 in [0, 2^32)
    long long c = l0 >> 32;
    l0 -= c * 4294967296LL;
    l1 += c;
    c = l1 >> 32;
    l1 -= c * 4294967296LL;
    l2 += c;
    const unsigned long long low = ((unsigned long long)l1 << 32) | (unsigned long long)l0;
    return (ldexp(double(l2), 64) + double(low)) * unscale;
}

template <typename FT>
__device__ __forceinline__ void ampere_edge(int ed, const FieldDesc &d)
{
    double ie;
    if (d.fx) {
        ie = fx_take(d.fx + 3 * size_t(ed), d.fx_unscale);
    } else {
        ie = d.cur[ed];
        d.cur[ed] = 0.0;
    }
    d.cur_last[ed] = ie;
    const int4 ef = d.edge_face[ed];
    if (ef.y < 0) return;  // wall edge: not a free DoF, d stays 0
    double curl = 0.0;
    curl += double(ef.z) * fget<FT>(d.h, ef.x);
    curl += double(ef.w) * fget<FT>(d.h, ef.y);
    double dn = d.d[ed] + d.dt * (curl - ie);
    if (d.damp) dn = dn * d.damp[ed];
    d.d[ed] = dn;
}

template <typename FT>
__global__ __launch_bounds__(256) void k_ampere(FieldDesc d)
{
    const int ed = blockIdx.x * blockDim.x + threadIdx.x;
    if (ed < d.ne) ampere_edge<FT>(ed, d);
}

// e = M~ d, M~ in SELL-64 (slices of 64 rows, column-major inside a slice;
// each row's entries in the column order of the CSR form).
template <typename FT>
__device__ __forceinline__ void spmv_row(int row, const FieldDesc &d)
{
    const int sl = row / kSlice, ln = row % kSlice;
    const int base = d.sl_ptr[sl], w = d.sl_w[sl];
    double acc = 0.0;
    if (d.pml_x) {
        // e = M~ (d + psi - phi) with the PML's auxiliary fluxes
        for (int j = 0; j < w; ++j) {
            const int q = base + j * kSlice + ln;
            const int c = d.sl_col[q];
            acc += fget<FT>(d.sl_val, q) * (d.d[c] + d.pml_x[c]);
        }
    } else {
        for (int j = 0; j < w; ++j) {
            const int q = base + j * kSlice + ln;
            acc += fget<FT>(d.sl_val, q) * d.d[d.sl_col[q]];
        }
    }
    fset<FT>(d.e_out, row, acc);
}

// Uniaxial PML along the layer normal n (stretching s = 1 + sigma/(j w
// eps0); permittivity eps0 diag(1/s, s) in (n, t)): per layer row k, from
// the current e, X = (M_n e)_k and Y = (M_t e)_k, then
//   psi <- (psi (1 - c/2) + c X) / (1 + c/2),  phi <- phi + c Y,
// c = kappa dt, and the SpMV takes e = M~ (d + psi - phi).
template <typename FT>
__device__ __forceinline__ void pml_row(int k, const FieldDesc &d)
{
    double x = 0.0, y = 0.0;
    for (int j = d.pn_ptr[k]; j < d.pn_ptr[k + 1]; ++j) x += d.pn_val[j] * fget<FT>(d.e, d.pn_col[j]);
    for (int j = d.pt_ptr[k]; j < d.pt_ptr[k + 1]; ++j) y += d.pt_val[j] * fget<FT>(d.e, d.pt_col[j]);
    const double c = d.pml_kappa[k] * d.dt;
    const double psi = (d.pml_psi[k] * (1.0 - 0.5 * c) + c * x) / (1.0 + 0.5 * c);
    const double phi = d.pml_phi[k] + c * y;
    d.pml_psi[k] = psi;
    d.pml_phi[k] = phi;
    d.pml_x[d.pml_rows[k]] = psi - phi;
}

template <typename FT>
__global__ __launch_bounds__(256) void k_pml_aux(FieldDesc d)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < d.pml_n) pml_row<FT>(k, d);
}

template <typename FT>
__global__ __launch_bounds__(256) void k_spmv(FieldDesc d)
{
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row < d.ne) spmv_row<FT>(row, d);
}

__global__ __launch_bounds__(256) void k_ampere_batched(const FieldDesc *__restrict__ runs,
                                                        const uint32_t *__restrict__ prefix,
                                                        int nrun, uint32_t total_blocks)
{
    for (uint32_t g = blockIdx.x; g < total_blocks; g += gridDim.x) {
        const int r = run_of(prefix, nrun, g);
        const FieldDesc &d = runs[r];
        const int ed = int(g - prefix[r]) * 256 + int(threadIdx.x);
        if (ed >= d.ne) continue;
        if (d.field32) ampere_edge<float>(ed, d);
        else ampere_edge<double>(ed, d);
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
        if (row >= d.ne) continue;
        if (d.field32) spmv_row<float>(row, d);
        else spmv_row<double>(row, d);
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
    const uint32_t h = a.tile_home[(blk * kSortB) / a.tile];
    return h > kSortBack ? h - kSortBack : 0u;
}

// Runs of equal in-window bins along a wavefront.  The particles are nearly
// sorted, so most of a wavefront's lanes share one or two bins; LDS atomics
// to one address from many lanes are serialised, so one lane per run (its
// head) adds the run's length.  Lanes outside the window or lost take a
// class of their own and form runs of one.  Returns the head mask; `len` is
// the run length on head lanes.
__device__ __forceinline__ uint64_t bin_runs(bool in, uint32_t bin, int lane, int &len)
{
    const uint32_t cls = in ? bin : 0x10000u + uint32_t(lane);
    const uint32_t prev = __shfl_up(cls, 1, 64);
    const bool head = lane == 0 || cls != prev;
    const uint64_t heads = __ballot(head);
    const uint64_t after = heads & ~((2ull << lane) - 1ull);
    len = (after ? __builtin_ctzll(after) : 64) - lane;
    return heads;
}

// The block's kSortPer keys per thread, all loads in flight at once (past
// the end: the lost key; the loads themselves stay in bounds).
__device__ __forceinline__ void load_block_keys(const SortArgs &a, int64_t b0,
                                                uint32_t (&key)[kSortPer])
{
#pragma unroll
    for (int j = 0; j < kSortPer; ++j) {
        const int64_t i = b0 + j * 256 + int(threadIdx.x);
        key[j] = a.key_in[i < a.n ? i : a.n - 1];
    }
#pragma unroll
    for (int j = 0; j < kSortPer; ++j)
        if (b0 + j * 256 + int(threadIdx.x) >= a.n) key[j] = kLost;
}

__global__ __launch_bounds__(256) void k_sort_hist(SortArgs a)
{
    __shared__ int32_t h[kSortBins];
    for (int t = threadIdx.x; t < kSortBins; t += 256) h[t] = 0;
    const uint32_t wb = sort_window(a, blockIdx.x);
    const int lane = threadIdx.x & 63;
    __syncthreads();
    const int64_t b0 = int64_t(blockIdx.x) * kSortB;
    uint32_t key[kSortPer];
    load_block_keys(a, b0, key);
#pragma unroll
    for (int j = 0; j < kSortPer; ++j) {
        const uint32_t k = key[j];
        const uint32_t f = k & kTriMask, bin = f - wb;
        const bool in = k != kLost && bin < uint32_t(kSortBins);
        int len;
        const uint64_t heads = bin_runs(in, bin, lane, len);
        if (in && ((heads >> lane) & 1ull)) atomicAdd(&h[bin], len);
        else if (k != kLost && !in) atomicAdd(a.counts + f, 1);
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
    uint32_t key[kSortPer];
    load_block_keys(a, b0, key);
#pragma unroll
    for (int j = 0; j < kSortPer; ++j) {
        const uint32_t k = key[j];
        const uint32_t f = k & kTriMask, b = f - wb;
        const bool in = k != kLost && b < uint32_t(kSortBins);
        // one LDS atomic per run of equal bins; the run's lanes take
        // consecutive ranks after the head's
        int len;
        const uint64_t heads = bin_runs(in, b, lane, len);
        const int head = 63 - __builtin_clzll(heads & ((2ull << lane) - 1ull));
        int base = 0;
        if (in && head == lane) base = atomicAdd(&cnt[b], len);
        base = __shfl(base, head, 64);
        bin[j] = -1;
        rank[j] = -1;
        if (k == kLost) continue;
        if (in) {
            bin[j] = int32_t(b);
            rank[j] = base + (lane - head);
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
    // (the four reservations are all in flight before their results are used)
    int32_t off4[4] = {0, 0, 0, 0}, at4[4] = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int b = 4 * tid + q;
        loc[b] = before;
        before += c4[q];
        if (c4[q]) {
            off4[q] = a.offsets[wb + uint32_t(b)];
            at4[q] = atomicAdd(a.counts + wb + uint32_t(b), c4[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) cnt[4 * tid + q] = off4[q] + at4[q];
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
    // (every slot's loads are in flight before the stores, which might
    // alias the inputs for all the compiler knows)
    const int n_in = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    const int nout = n_out;
    const E *lam_in = reinterpret_cast<const E *>(a.lam_in);
    const E *u_in = reinterpret_cast<const E *>(a.u_in);
    E *lam_out = reinterpret_cast<E *>(a.lam_out);
    E *u_out = reinterpret_cast<E *>(a.u_out);
    constexpr int kGroup = 8;
    static_assert(kSortPer % kGroup == 0, "copy groups");
#pragma unroll
    for (int g = 0; g < kSortPer; g += kGroup) {
        bool on[kGroup];
        int32_t dst[kGroup];
        uint32_t kv[kGroup], pv[kGroup];
        E lv[kGroup], uv[kGroup];
#pragma unroll
        for (int q = 0; q < kGroup; ++q) {
            // loads without a branch (an empty slot reads the block's first
            // particle and stores nothing), so the group's loads stay in flight
            const int s = (g + q) * 256 + tid;
            on[q] = s < n_in || s >= kSortB - nout;
            const int64_t src = b0 + (on[q] ? s_src[s] : 0);
            dst[q] = s_dst[s];
            kv[q] = a.key_in[src];
            lv[q] = lam_in[src];
            uv[q] = u_in[src];
            pv[q] = a.pid_in[src];
        }
        // every loaded value counts as used here, so the compiler cannot sink
        // the loads into the conditional stores below, one slot at a time
#pragma unroll
        for (int q = 0; q < kGroup; ++q)
            asm volatile("" ::"v"(kv[q]), "v"(pv[q]), "v"(lv[q].x), "v"(lv[q].y), "v"(uv[q].x),
                         "v"(uv[q].y));
#pragma unroll
        for (int q = 0; q < kGroup; ++q) {
            if (!on[q]) continue;
            a.key_out[dst[q]] = kv[q];
            lam_out[dst[q]] = lv[q];
            u_out[dst[q]] = uv[q];
            a.pid_out[dst[q]] = pv[q];
        }
    }
}

// p[i] = v for offsets start[0] <= i < n (a grid-stride loop over a fixed
// grid: the start is known only on the device).
constexpr int kTailBlocks = 1024;
__global__ __launch_bounds__(256) void k_fill_tail(uint32_t *__restrict__ p,
                                                   const int32_t *__restrict__ start, int64_t n,
                                                   uint32_t v)
{
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(*start) + int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += stride)
        p[i] = v;
}

// Home triangle of every tile of the sorted segment (its first particle).
__global__ __launch_bounds__(256) void k_tile_home(int64_t n, const uint32_t *__restrict__ key,
                                                   uint32_t *__restrict__ home, int64_t tiles,
                                                   int64_t tile)
{
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= tiles) return;
    const int64_t i = t * tile;
    const uint32_t k = i < n ? key[i] : kLost;
    home[t] = k == kLost ? 0u : (k & kTriMask);
}

// ---------------------------------------------------------------------
// Field probes: E = sum_k s_k e_k (l_a grad l_b - l_b grad l_a) (Sec. II.B)
// at fixed points, accumulated over a window of steps; at the end of a
// window the average is written out and the sum restarts.
// ---------------------------------------------------------------------
template <typename FT>
__global__ __launch_bounds__(256) void k_probe(int n, const int32_t *__restrict__ tri,
                                               const double *__restrict__ lam,
                                               const int4 *__restrict__ tri_edge,
                                               const double *__restrict__ grad,
                                               const FT *__restrict__ e,
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
    const double e0 = double(e[te.x]), e1 = double(e[te.y]), e2 = double(e[te.z]);
    const double s0 = (te.w & 1) ? -e0 : e0;
    const double s1 = (te.w & 2) ? -e1 : e1;
    const double s2 = (te.w & 4) ? -e2 : e2;
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

// Plain 16-byte-vector copy, grid-stride: the achievable HBM bandwidth of a
// stream that reads and writes every byte once (the reference ceiling the
// particle kernel is compared with).
__global__ __launch_bounds__(256) void k_copy(const float4 *__restrict__ src,
                                              float4 *__restrict__ dst, int64_t n)
{
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

}  // namespace

hipError_t launch_copy(hipStream_t s, const void *src, void *dst, int64_t n16, int blocks)
{
    if (n16 <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, static_cast<const float4 *>(src),
                       static_cast<float4 *>(dst), n16);
    return hipGetLastError();
}

hipError_t launch_faraday(hipStream_t s, const FieldDesc &d)
{
    if (d.nf <= 0) return hipSuccess;
    if (d.field32) FETD_LAUNCH(k_faraday<float>, dim3(grid_for(d.nf, 256)), dim3(256), 0, s, d);
    else FETD_LAUNCH(k_faraday<double>, dim3(grid_for(d.nf, 256)), dim3(256), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_ampere(hipStream_t s, const FieldDesc &d)
{
    if (d.ne <= 0) return hipSuccess;
    if (d.field32) FETD_LAUNCH(k_ampere<float>, dim3(grid_for(d.ne, 256)), dim3(256), 0, s, d);
    else FETD_LAUNCH(k_ampere<double>, dim3(grid_for(d.ne, 256)), dim3(256), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_spmv(hipStream_t s, const FieldDesc &d)
{
    if (d.ne <= 0) return hipSuccess;
    if (d.field32) FETD_LAUNCH(k_spmv<float>, dim3(grid_for(d.ne, 256)), dim3(256), 0, s, d);
    else FETD_LAUNCH(k_spmv<double>, dim3(grid_for(d.ne, 256)), dim3(256), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_pml_aux(hipStream_t s, const FieldDesc &d)
{
    if (d.pml_n <= 0) return hipSuccess;
    if (d.field32) FETD_LAUNCH(k_pml_aux<float>, dim3(grid_for(d.pml_n, 256)), dim3(256), 0, s, d);
    else FETD_LAUNCH(k_pml_aux<double>, dim3(grid_for(d.pml_n, 256)), dim3(256), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_probe(hipStream_t s, int n, const int32_t *tri, const double *lam,
                        const int4 *tri_edge, const double *grad64, const void *e, bool field32,
                        double *acc, double *out, double inv_window)
{
    if (n <= 0) return hipSuccess;
    if (field32)
        hipLaunchKernelGGL(k_probe<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, n, tri, lam,
                           tri_edge, grad64, static_cast<const float *>(e), acc, out, inv_window);
    else
        hipLaunchKernelGGL(k_probe<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, n, tri, lam,
                           tri_edge, grad64, static_cast<const double *>(e), acc, out, inv_window);
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
    if (a.n > 0)
        hipLaunchKernelGGL(k_sort_hist, dim3(grid_for(a.n, kSortB)), dim3(256), 0, s, a);
    const int nb = int((a.nf + 1023) / 1024);
    hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(1024), 0, s, a.nf, a.counts, a.offsets,
                       a.block_sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, nb, a.block_sums);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(1024), 0, s, a.nf, a.offsets, a.block_sums, nb);
    // slots past the live count (offsets[nf]) hold the lost key
    if (a.n > 0)
        hipLaunchKernelGGL(k_fill_tail, dim3(kTailBlocks), dim3(256), 0, s, a.key_out,
                           a.offsets + a.nf, a.n, kLost);
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
        err = launch_tile_home(s, a.n, a.key_out, a.tile_home, a.tile);
        if (err != hipSuccess) return err;
    }
    return hipGetLastError();
}

hipError_t launch_tile_home(hipStream_t s, int64_t n, const uint32_t *key, uint32_t *home,
                            int64_t tile)
{
    if (n <= 0) return hipSuccess;
    if (tile < kBlock) return hipErrorInvalidValue;
    const int64_t tiles = (n + tile - 1) / tile;
    hipLaunchKernelGGL(k_tile_home, dim3(grid_for(tiles, 256)), dim3(256), 0, s, n, key, home,
                       tiles, tile);
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
