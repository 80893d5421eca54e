/*
 * FP64 CPU oracle for the relativistic charge-conserving FETD-PIC step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, single-threaded
 * statement of what one PIC step computes, written from the paper
 * (Na, Moon, Omelchenko, Teixeira, "Relativistic extension of a
 * charge-conservative finite element solver for time-dependent
 * Maxwell-Vlasov equations", arXiv:1707.04333).  Only the test-suite, the
 * smoke check and the CPU baseline of the benchmark may load it.  It shares
 * no code with the HIP library.
 *
 * Conventions (the paper leaves them open; the readings are the ones the
 * tests pin):
 *   - triangles are counter-clockwise; local edge k is opposite local
 *     node k and runs from local node a=(k+1)%3 to b=(k+2)%3;
 *   - a global edge is oriented from its lower to its higher node id;
 *     sign(f,k) = +1 when a->b matches that orientation;
 *   - grad lambda_k = perp(x_b - x_a) / (2A), perp(x,y) = (-y, x);
 *   - a particle stores its triangle, a "derived slot" r and the
 *     barycentric pair of local nodes (r+1)%3, (r+2)%3; the third
 *     coordinate is (1 - l_{r+1}) - l_{r+2};
 *   - the field state is d = [*eps] e (FP64), e = M~ d with M~ the
 *     approximate inverse of [*eps]; b holds face fluxes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nf, ne, nn;
    const int32_t *tri_node;   /* [3nf] */
    const int32_t *tri_edge;   /* [3nf] */
    const int8_t *tri_sign;    /* [3nf] +1 / -1 */
    const int32_t *tri_nbr;    /* [3nf] neighbour across local edge k, <0 = wall */
    const int8_t *tri_nbrk;    /* [3nf] local index of the shared edge in the neighbour */
    const double *vxy;         /* [6nf] image-consistent vertex coordinates */
    const double *grad;        /* [6nf] grad lambda_k (x, y) per local node */
    const double *area;        /* [nf] */
    const int32_t *edge_tri;   /* [2ne] adjacent triangles, -1 if none */
    const int8_t *edge_tsign;  /* [2ne] sign of the edge in that triangle */
    const uint8_t *edge_free;  /* [ne] */
    const int32_t *mt_ptr;     /* CSR of the approximate inverse M~ */
    const int32_t *mt_col;
    const double *mt_val;
} o_mesh;

enum { O_BORIS = 0, O_BORIS_TAN = 1, O_VAY = 2, O_HC = 3 };

/* ---------------------------------------------------------------------- */
/* Pushers, written for general 3-vectors (Sec. II.C).                    */
/* ---------------------------------------------------------------------- */

static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double *a, const double *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* gamma(u) = sqrt(1 + |u|^2/c^2) with u = gamma v (Sec. II.C). */
static double gamma_of(const double *u, double c)
{
    return sqrt(1.0 + dot3(u, u) / (c * c));
}

/*
 * One momentum update u^{n-1/2} -> u^{n+1/2} (Sec. II.C, eqs.
 * Lorentz.Newton.dis and Boris.u1-u4).  eps = alpha E^n, beta = alpha B^n,
 * alpha = q dt / (2 m0).
 *
 * Boris: u- = u + eps; gbar = gamma(u-) (eq. gamma.middle); t = beta/gbar;
 *   s = 2t/(1+|t|^2); u' = u- + u- x t; u+ = u- + u' x s; u = u+ + eps.
 * Boris with tan correction: t = (beta/|beta|) tan(|beta|/gbar).
 * Vay (Sec. II.C(b)), read as the exact solution of its implicit midpoint
 *   equation u+ = u' + (u+/gamma+) x beta: u_h = u + eps + v x beta,
 *   u' = u_h + eps, sigma = gamma(u')^2 - |beta|^2, u* = u'.beta/c,
 *   gamma+ = sqrt((sigma + sqrt(sigma^2 + 4(|beta|^2 + u*^2)))/2),
 *   t = beta/gamma+, s = 1/(1+|t|^2), u = s[u' + (u'.t)t + u' x t].
 * Higuera-Cary (Sec. II.C(c)): Boris rotation with gbar replaced by
 *   gamma_H = sqrt((sigma + sqrt(sigma^2 + 4(|beta|^2 + w^2)))/2),
 *   sigma = gamma(u-)^2 - |beta|^2, w = beta.u-/c.
 */
void o_push(int pusher, const double *u, const double *eps, const double *beta,
            double c, double *out)
{
    double um[3], t[3], s[3], up[3], tmp[3];
    if (pusher == O_VAY) {
        double g = gamma_of(u, c);
        double v[3] = {u[0] / g, u[1] / g, u[2] / g};
        cross3(v, beta, tmp);
        double uh[3], upr[3];
        for (int i = 0; i < 3; ++i) uh[i] = u[i] + eps[i] + tmp[i];
        for (int i = 0; i < 3; ++i) upr[i] = uh[i] + eps[i];
        double gp = gamma_of(upr, c);
        double bb = dot3(beta, beta);
        double sig = gp * gp - bb;
        double us = dot3(upr, beta) / c;
        double gn = sqrt(0.5 * (sig + sqrt(sig * sig + 4.0 * (bb + us * us))));
        for (int i = 0; i < 3; ++i) t[i] = beta[i] / gn;
        double sv = 1.0 / (1.0 + dot3(t, t));
        double ut = dot3(upr, t);
        cross3(upr, t, tmp);
        for (int i = 0; i < 3; ++i) out[i] = sv * (upr[i] + ut * t[i] + tmp[i]);
        return;
    }
    for (int i = 0; i < 3; ++i) um[i] = u[i] + eps[i];
    double gbar;
    if (pusher == O_HC) {
        double bb = dot3(beta, beta);
        double gm = gamma_of(um, c);
        double sig = gm * gm - bb;
        double w = dot3(beta, um) / c;
        gbar = sqrt(0.5 * (sig + sqrt(sig * sig + 4.0 * (bb + w * w))));
    } else {
        gbar = gamma_of(um, c);
    }
    if (pusher == O_BORIS_TAN) {
        double bm = sqrt(dot3(beta, beta));
        if (bm > 0.0) {
            double f = tan(bm / gbar) / bm;
            for (int i = 0; i < 3; ++i) t[i] = beta[i] * f;
        } else {
            t[0] = t[1] = t[2] = 0.0;
        }
    } else {
        for (int i = 0; i < 3; ++i) t[i] = beta[i] / gbar;
    }
    double tt = dot3(t, t);
    for (int i = 0; i < 3; ++i) s[i] = 2.0 * t[i] / (1.0 + tt);
    cross3(um, t, tmp);
    for (int i = 0; i < 3; ++i) up[i] = um[i] + tmp[i];
    cross3(up, s, tmp);
    for (int i = 0; i < 3; ++i) out[i] = um[i] + tmp[i] + eps[i];
}

/* ---------------------------------------------------------------------- */
/* Gather (Sec. II.B): E = sum_i e_i W1_i(r_p), B = sum_i b_i W2_i(r_p).    */
/* ---------------------------------------------------------------------- */

static void local_lambda(int r, const double *pair, double *L)
{
    int p = (r + 1) % 3, q = (r + 2) % 3;
    L[p] = pair[0];
    L[q] = pair[1];
    L[r] = (1.0 - pair[0]) - pair[1];
}

/* Whitney 1-form of local edge k: W = l_a grad l_b - l_b grad l_a. */
void o_gather_e(const o_mesh *M, const double *e, const double *e_ext, int f,
                const double *L, double *E)
{
    const double *G = M->grad + 6 * f;
    double ex = 0.0, ey = 0.0;
    for (int k = 0; k < 3; ++k) {
        int a = (k + 1) % 3, b = (k + 2) % 3;
        int ed = M->tri_edge[3 * f + k];
        double dof = e[ed];
        if (e_ext) dof = dof + e_ext[ed];
        double s = M->tri_sign[3 * f + k] * dof;
        ex += s * (L[a] * G[2 * b] - L[b] * G[2 * a]);
        ey += s * (L[a] * G[2 * b + 1] - L[b] * G[2 * a + 1]);
    }
    E[0] = ex;
    E[1] = ey;
}

/* ---------------------------------------------------------------------- */
/* Scatter (Sec. II.D, eq. I.assign): current of one straight segment     */
/* inside triangle f, from barycentrics Ls to Lf.                          */
/* ---------------------------------------------------------------------- */

static void deposit_segment(const o_mesh *M, int f, const double *Ls, const double *Lf,
                            double qdt, double *cur)
{
    for (int k = 0; k < 3; ++k) {
        int a = (k + 1) % 3, b = (k + 2) % 3;
        double w = Ls[a] * Lf[b] - Lf[a] * Ls[b];
        cur[M->tri_edge[3 * f + k]] += M->tri_sign[3 * f + k] * qdt * w;
    }
}

/*
 * Move one particle by dr inside the mesh, splitting the straight path at
 * triangle edges and depositing each piece (the exact current of eq.
 * I.assign holds inside one triangle).  Returns the number of segments, or
 * -1 when the crossing cap is exceeded.  *lost is set when the path meets
 * a wall; the current up to the wall is deposited.
 *
 * Exit rule (our reading; the paper defers tracking to its refs): with
 * dL_k = grad l_k . dr_rem, the candidates are the local edges k with
 * dL_k < 0, excluding the edge just entered; tau_k = max(l_k,0)/(-dL_k);
 * the smallest tau wins, ties to the smallest k.  tau >= 1 ends inside.
 * At an exit through edge k the point has l_k = 0, l_a = l_a + tau dL_a and
 * l_b = 1 - l_a; the neighbour inherits l_a, l_b by node identity.
 *
 * seg_tri / seg_L (optional, capacity cap) record the path.
 */
int o_move(const o_mesh *M, int32_t *ptri, int8_t *pslot, double *pair, double dx,
           double dy, double qdt, double *cur, int cap, int *lost, int32_t *seg_tri,
           double *seg_L)
{
    int f = *ptri, r = *pslot;
    double L[3], Lf[3];
    local_lambda(r, pair, L);
    int entry = -1;
    double rx = dx, ry = dy;
    *lost = 0;
    for (int it = 0; it < cap; ++it) {
        const double *G = M->grad + 6 * f;
        double dL[3];
        for (int k = 0; k < 3; ++k) dL[k] = G[2 * k] * rx + G[2 * k + 1] * ry;
        int ks = -1;
        double ts = 0.0;
        for (int k = 0; k < 3; ++k) {
            if (k == entry || !(dL[k] < 0.0)) continue;
            double tk = (L[k] > 0.0 ? L[k] : 0.0) / (-dL[k]);
            if (ks < 0 || tk < ts) {
                ks = k;
                ts = tk;
            }
        }
        if (ks < 0 || ts >= 1.0) {
            int p = (r + 1) % 3, q = (r + 2) % 3;
            double np_ = L[p] + dL[p];
            double nq = L[q] + dL[q];
            Lf[p] = np_;
            Lf[q] = nq;
            Lf[r] = (1.0 - np_) - nq;
            deposit_segment(M, f, L, Lf, qdt, cur);
            if (seg_tri) {
                seg_tri[it] = f;
                memcpy(seg_L + 6 * it, L, sizeof L);
                memcpy(seg_L + 6 * it + 3, Lf, sizeof Lf);
            }
            *ptri = f;
            *pslot = (int8_t)r;
            pair[0] = np_;
            pair[1] = nq;
            return it + 1;
        }
        int a = (ks + 1) % 3, b = (ks + 2) % 3;
        double la = L[a] + ts * dL[a];
        Lf[ks] = 0.0;
        Lf[a] = la;
        Lf[b] = 1.0 - la;
        deposit_segment(M, f, L, Lf, qdt, cur);
        if (seg_tri) {
            seg_tri[it] = f;
            memcpy(seg_L + 6 * it, L, sizeof L);
            memcpy(seg_L + 6 * it + 3, Lf, sizeof Lf);
        }
        int nb = M->tri_nbr[3 * f + ks];
        if (nb < 0) {
            /* Wall: the particle leaves the domain at the exit point. */
            *lost = 1;
            *ptri = f;
            *pslot = (int8_t)b;
            pair[0] = 0.0; /* local (b+1)%3 = ks */
            pair[1] = la;  /* local (b+2)%3 = a  */
            return it + 1;
        }
        int kk = M->tri_nbrk[3 * f + ks];
        int a2 = (kk + 1) % 3, b2 = (kk + 2) % 3;
        /* CCW neighbours traverse the shared edge in opposite directions:
           node a of f is node b2 of nb, node b of f is node a2 of nb. */
        L[kk] = 0.0;
        L[b2] = la;
        L[a2] = 1.0 - la;
        r = a2;
        f = nb;
        entry = kk;
        double sc = 1.0 - ts;
        rx = rx * sc;
        ry = ry * sc;
    }
    return -1;
}

/* ---------------------------------------------------------------------- */
/* Field update (Sec. II.A, eqs. semi.dis.curl.1/2).                       */
/* ---------------------------------------------------------------------- */

/* b^{n+1/2} = b^{n-1/2} - dt C e^n.  damp_b (optional) multiplies b on
 * absorbing-layer triangles after the update: the magnetic loss that
 * matches the layer's electric conductivity (sigma_m / mu0 = sigma / eps0,
 * the same factor as on d). */
void o_faraday(const o_mesh *M, const double *b_old, const double *e, double dt,
               const double *damp_b, double *b_new)
{
    for (int f = 0; f < M->nf; ++f) {
        double circ = 0.0;
        for (int k = 0; k < 3; ++k)
            circ += M->tri_sign[3 * f + k] * e[M->tri_edge[3 * f + k]];
        b_new[f] = b_old[f] - dt * circ;
        if (damp_b) b_new[f] = b_new[f] * damp_b[f];
    }
}

/*
 * d^{n+1} = d^n + dt (C^T [*mu^-1] b^{n+1/2} - i^{n+1/2}) on free edges,
 * then e^{n+1} = M~ d^{n+1}.  [*mu^-1] = diag(1/(mu0 A_f)) for the face
 * 2-forms W2_f = z/A_f.  damp (optional) multiplies d on absorbing-layer
 * edges after the update.  Non-free (wall) edges keep d = e = 0.
 */
void o_ampere(const o_mesh *M, const double *b_half, const double *cur, double dt,
              double mu0, const double *damp, double *d, double *e)
{
    for (int ed = 0; ed < M->ne; ++ed) {
        if (!M->edge_free[ed]) {
            d[ed] = 0.0;
            continue;
        }
        double curl = 0.0;
        for (int j = 0; j < 2; ++j) {
            int f = M->edge_tri[2 * ed + j];
            if (f < 0) continue;
            curl += M->edge_tsign[2 * ed + j] * (b_half[f] / (mu0 * M->area[f]));
        }
        d[ed] = d[ed] + dt * (curl - cur[ed]);
        if (damp) d[ed] = d[ed] * damp[ed];
    }
    for (int ed = 0; ed < M->ne; ++ed) {
        if (!M->edge_free[ed]) {
            e[ed] = 0.0;
            continue;
        }
        double acc = 0.0;
        for (int j = M->mt_ptr[ed]; j < M->mt_ptr[ed + 1]; ++j)
            acc += M->mt_val[j] * d[M->mt_col[j]];
        e[ed] = acc;
    }
}

/* ---------------------------------------------------------------------- */
/* Particle stage of one step for one species: gather, push, move, track,  */
/* deposit.  Particles with tri < 0 are lost and skipped.                  */
/* Returns 0, or -1 (crossing cap) / -2 (non-finite momentum) with *bad    */
/* the first offending particle.  counts[0] += segments, counts[1] += lost */
/* seq / nseq (optional): the triangle of each straight piece of particle  */
/* p's move, the first seqcap of them at seq[p * seqcap], and the number   */
/* of pieces in nseq[p] (0 for a particle lost before the step).           */
/* ---------------------------------------------------------------------- */
int o_particles(const o_mesh *M, const double *e, const double *e_ext,
                const double *b_old, const double *b_new, const double *bz_ext,
                const double *affine, int pusher, double q, double m, double w,
                double dt, double c, int cap, int64_t n, int32_t *tri, int8_t *slot,
                double *lam, double *u, double *cur, int64_t *counts, int64_t *bad,
                int32_t *seq, int seqcap, int32_t *nseq)
{
    double alpha = q * dt / (2.0 * m);
    double qdt = q * w / dt;
    int32_t *seg_tri = NULL;
    double *seg_L = NULL;
    if (seq) {
        seg_tri = malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
        seg_L = malloc(sizeof(double) * 6 * (size_t)(cap > 0 ? cap : 1));
        if (!seg_tri || !seg_L) {
            free(seg_tri);
            free(seg_L);
            return -3;
        }
    }
    int rc = 0;
    for (int64_t p = 0; p < n; ++p) {
        int f = tri[p];
        if (nseq) nseq[p] = 0;
        if (f < 0) continue;
        double L[3];
        local_lambda(slot[p], lam + 2 * p, L);
        double E[3] = {0.0, 0.0, 0.0};
        o_gather_e(M, e, e_ext, f, L, E);
        if (affine) {
            const double *v = M->vxy + 6 * f;
            double x = L[0] * v[0] + L[1] * v[2] + L[2] * v[4];
            double y = L[0] * v[1] + L[1] * v[3] + L[2] * v[5];
            E[0] += affine[0] + affine[2] * x + affine[3] * y;
            E[1] += affine[1] + affine[4] * x + affine[5] * y;
        }
        /* B^n = (B^{n+1/2} + B^{n-1/2})/2 at r^n (Sec. II.C); W2_f = z/A_f. */
        double bz = (b_new[f] + b_old[f]) / (2.0 * M->area[f]);
        if (bz_ext) bz += bz_ext[f];
        double eps[3] = {alpha * E[0], alpha * E[1], 0.0};
        double beta[3] = {0.0, 0.0, alpha * bz};
        double u0[3] = {u[2 * p], u[2 * p + 1], 0.0};
        double u1[3];
        o_push(pusher, u0, eps, beta, c, u1);
        if (!isfinite(u1[0]) || !isfinite(u1[1])) {
            *bad = p;
            rc = -2;
            break;
        }
        u[2 * p] = u1[0];
        u[2 * p + 1] = u1[1];
        /* r^{n+1} = r^n + dt u^{n+1/2} / gamma^{n+1/2} (eq. eq.motion.dis). */
        double g = gamma_of(u1, c);
        double dx = dt * u1[0] / g;
        double dy = dt * u1[1] / g;
        int32_t t32 = f;
        int8_t s8 = slot[p];
        int lost = 0;
        int ns = o_move(M, &t32, &s8, lam + 2 * p, dx, dy, qdt, cur, cap, &lost, seg_tri, seg_L);
        if (ns < 0) {
            *bad = p;
            rc = -1;
            break;
        }
        if (seq) {
            for (int k = 0; k < ns && k < seqcap; ++k) seq[p * seqcap + k] = seg_tri[k];
            nseq[p] = ns;
        }
        counts[0] += ns;
        if (lost) {
            counts[1] += 1;
            tri[p] = -1;
        } else {
            tri[p] = t32;
        }
        slot[p] = s8;
    }
    free(seg_tri);
    free(seg_L);
    return rc;
}

/* Nodal charge q_i = sum_p Q lambda_i(r_p) (Sec. II.D, eq.
   scatter.charge.assign), accumulated into qn[nn]. */
void o_charge(const o_mesh *M, double qw, int64_t n, const int32_t *tri,
              const int8_t *slot, const double *lam, double *qn)
{
    for (int64_t p = 0; p < n; ++p) {
        int f = tri[p];
        if (f < 0) continue;
        double L[3];
        local_lambda(slot[p], lam + 2 * p, L);
        for (int k = 0; k < 3; ++k) qn[M->tri_node[3 * f + k]] += qw * L[k];
    }
}

/* ---------------------------------------------------------------------- */
/* Sparse approximate inverse (Sec. II.A): for every column j minimise     */
/* || M m_j - e_j ||_2 over the sparsity pattern of column j of the k-th   */
/* power of M's graph (Frobenius-norm SPAI), then symmetrise.              */
/* Solves each small least-squares problem by Householder QR.              */
/* ---------------------------------------------------------------------- */

static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* Least squares min ||A x - rhs|| for A (m x n, column-major, m >= n). */
static void lstsq_householder(double *A, int m, int n, double *rhs, double *x)
{
    for (int j = 0; j < n; ++j) {
        double *col = A + (size_t)j * m;
        double nrm = 0.0;
        for (int i = j; i < m; ++i) nrm += col[i] * col[i];
        nrm = sqrt(nrm);
        if (nrm == 0.0) continue;
        double alpha = col[j] > 0 ? -nrm : nrm;
        double v0 = col[j] - alpha;
        /* v = (v0, col[j+1..]) ; H = I - 2 v v^T / (v^T v) */
        double vtv = v0 * v0;
        for (int i = j + 1; i < m; ++i) vtv += col[i] * col[i];
        for (int c2 = j + 1; c2 < n; ++c2) {
            double *cc = A + (size_t)c2 * m;
            double s = v0 * cc[j];
            for (int i = j + 1; i < m; ++i) s += col[i] * cc[i];
            s = 2.0 * s / vtv;
            cc[j] -= s * v0;
            for (int i = j + 1; i < m; ++i) cc[i] -= s * col[i];
        }
        double s = v0 * rhs[j];
        for (int i = j + 1; i < m; ++i) s += col[i] * rhs[i];
        s = 2.0 * s / vtv;
        rhs[j] -= s * v0;
        for (int i = j + 1; i < m; ++i) rhs[i] -= s * col[i];
        col[j] = alpha;
    }
    for (int j = n - 1; j >= 0; --j) {
        double s = rhs[j];
        for (int c2 = j + 1; c2 < n; ++c2) s -= A[(size_t)c2 * m + j] * x[c2];
        double dgn = A[(size_t)j * m + j];
        x[j] = dgn != 0.0 ? s / dgn : 0.0;
    }
}

/* Pattern of column j: nodes within `level` hops of j in the graph of M. */
static int pattern(int n, const int32_t *ptr, const int32_t *col, int j, int level,
                   int *mark, int stamp, int *out, int cap)
{
    int cnt = 0, head = 0;
    out[cnt++] = j;
    mark[j] = stamp;
    for (int l = 0; l < level; ++l) {
        int end = cnt;
        for (; head < end; ++head) {
            int v = out[head];
            for (int q = ptr[v]; q < ptr[v + 1]; ++q) {
                int w = col[q];
                if (mark[w] != stamp) {
                    if (cnt >= cap) return -1;
                    mark[w] = stamp;
                    out[cnt++] = w;
                }
            }
        }
    }
    (void)n;
    qsort(out, cnt, sizeof(int), cmp_int);
    return cnt;
}

/*
 * Build the SPAI of the symmetric sparse M (CSR, n x n).  Output CSR with
 * the symmetric pattern; out_ptr has n+1 entries, out_col/out_val have
 * capacity `cap_nnz`.  Returns nnz, or -1 on overflow.
 */
int64_t o_spai(int n, const int32_t *ptr, const int32_t *col, const double *val, int level,
               int32_t *out_ptr, int32_t *out_col, double *out_val, int64_t cap_nnz)
{
    const int PCAP = 4096;
    int *mark = calloc((size_t)n, sizeof(int));
    int *rmark = calloc((size_t)n, sizeof(int));
    int *rpos = malloc((size_t)n * sizeof(int));
    int *J = malloc(PCAP * sizeof(int));
    int *I = malloc(PCAP * 8 * sizeof(int));
    double *A = malloc((size_t)PCAP * 8 * 64 * sizeof(double));
    double *rhs = malloc(PCAP * 8 * sizeof(double));
    double *x = malloc(PCAP * sizeof(double));
    /* column solutions stored CSC-like with the same pattern */
    int32_t *cptr = malloc(((size_t)n + 1) * sizeof(int32_t));
    int64_t nnz = 0;
    cptr[0] = 0;
    int64_t ok = 0;
    for (int j = 0; j < n; ++j) {
        int nj = pattern(n, ptr, col, j, level, mark, j + 1, J, PCAP);
        if (nj < 0 || nj > 64 || nnz + nj > cap_nnz) {
            ok = -1;
            break;
        }
        int ni = 0;
        for (int a = 0; a < nj; ++a) {
            int cj = J[a];
            for (int q = ptr[cj]; q < ptr[cj + 1]; ++q) {
                int r = col[q];
                if (rmark[r] != j + 1) {
                    rmark[r] = j + 1;
                    I[ni++] = r;
                }
            }
        }
        qsort(I, ni, sizeof(int), cmp_int);
        for (int a = 0; a < ni; ++a) rpos[I[a]] = a;
        memset(A, 0, (size_t)ni * nj * sizeof(double));
        for (int a = 0; a < nj; ++a) {
            int cj = J[a];
            /* column cj of M = row cj of M (symmetric) */
            for (int q = ptr[cj]; q < ptr[cj + 1]; ++q) A[(size_t)a * ni + rpos[col[q]]] = val[q];
        }
        for (int a = 0; a < ni; ++a) rhs[a] = (I[a] == j) ? 1.0 : 0.0;
        lstsq_householder(A, ni, nj, rhs, x);
        for (int a = 0; a < nj; ++a) {
            out_col[nnz + a] = J[a];
            out_val[nnz + a] = x[a];
        }
        nnz += nj;
        cptr[j + 1] = (int32_t)nnz;
    }
    if (ok == 0) {
        /* Symmetrise: M~_ij = (m_ij + m_ji)/2; pattern is symmetric. */
        double *sym = malloc((size_t)nnz * sizeof(double));
        for (int j = 0; j < n; ++j) {
            for (int64_t q = cptr[j]; q < cptr[j + 1]; ++q) {
                int i = out_col[q];
                /* find j in column i */
                int lo = cptr[i], hi = cptr[i + 1] - 1;
                double mji = 0.0;
                while (lo <= hi) {
                    int mid = (lo + hi) / 2;
                    if (out_col[mid] == j) {
                        mji = out_val[mid];
                        break;
                    }
                    if (out_col[mid] < j) lo = mid + 1;
                    else hi = mid - 1;
                }
                sym[q] = 0.5 * (out_val[q] + mji);
            }
        }
        memcpy(out_val, sym, (size_t)nnz * sizeof(double));
        free(sym);
        for (int j = 0; j <= n; ++j) out_ptr[j] = cptr[j];
        ok = nnz;
    }
    free(mark);
    free(rmark);
    free(rpos);
    free(J);
    free(I);
    free(A);
    free(rhs);
    free(x);
    free(cptr);
    return ok;
}

/* ---------------------------------------------------------------------- */
/* Timing mode: the particle stage of o_particles spread over nthreads      */
/* OpenMP threads.  The particles are cut into nthreads contiguous chunks;  */
/* each thread runs o_particles on its chunk with a private current array,  */
/* and the private arrays are added into cur in thread order (a fixed        */
/* order: the result does not depend on scheduling, though its rounding     */
/* differs from the single-threaded sum).  Used to time the oracle on all   */
/* host cores; parity runs use o_particles.  Returns as o_particles; on an  */
/* error the first failing chunk's code and particle are reported.          */
/* ---------------------------------------------------------------------- */
int o_particles_omp(int nthreads, const o_mesh *M, const double *e, const double *e_ext,
                    const double *b_old, const double *b_new, const double *bz_ext,
                    const double *affine, int pusher, double q, double m, double w,
                    double dt, double c, int cap, int64_t n, int32_t *tri, int8_t *slot,
                    double *lam, double *u, double *cur, int64_t *counts, int64_t *bad,
                    int32_t *seq, int seqcap, int32_t *nseq)
{
    if (nthreads < 1) nthreads = 1;
    double *priv = calloc((size_t)nthreads * (size_t)M->ne, sizeof(double));
    int64_t *pc = calloc((size_t)nthreads * 2, sizeof(int64_t));
    int64_t *pbad = calloc((size_t)nthreads, sizeof(int64_t));
    int *prc = calloc((size_t)nthreads, sizeof(int));
    if (!priv || !pc || !pbad || !prc) {
        free(priv);
        free(pc);
        free(pbad);
        free(prc);
        return -3;
    }
#pragma omp parallel for num_threads(nthreads) schedule(static, 1)
    for (int t = 0; t < nthreads; ++t) {
        int64_t lo = n * t / nthreads, hi = n * (t + 1) / nthreads;
        prc[t] = o_particles(M, e, e_ext, b_old, b_new, bz_ext, affine, pusher, q, m, w, dt, c,
                             cap, hi - lo, tri + lo, slot + lo, lam + 2 * lo, u + 2 * lo,
                             priv + (size_t)t * M->ne, pc + 2 * t, pbad + t,
                             seq ? seq + lo * seqcap : NULL, seqcap, nseq ? nseq + lo : NULL);
        if (prc[t] != 0) pbad[t] += lo;
    }
    int rc = 0;
    for (int t = 0; t < nthreads; ++t) {
        for (int ed = 0; ed < M->ne; ++ed) cur[ed] += priv[(size_t)t * M->ne + ed];
        counts[0] += pc[2 * t];
        counts[1] += pc[2 * t + 1];
        if (rc == 0 && prc[t] != 0) {
            rc = prc[t];
            *bad = pbad[t];
        }
    }
    free(priv);
    free(pc);
    free(pbad);
    free(prc);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* Uniaxial perfectly matched layer (the absorbing boundary of Sec. III.C; */
/* the construction is the build's own, the paper's references are not     */
/* available).  For a layer stretched along axis n (s = 1 + sigma/(j w      */
/* eps0)), the permittivity tensor is eps0 diag(1/s, s) in (n, t) and the   */
/* permeability mu0 s.  Splitting the Hodge matrix [*eps] = M_n + M_t into   */
/* the parts of the two field components (int W_i,n W_j,n and               */
/* int W_i,t W_j,t) and taking the stretching per edge row                  */
/* (kappa = sigma_edge / eps0), the update of d = C^T [*mu^-1] b - i stays   */
/* that of the lossless medium, and                                         */
/*   e = [*eps]^-1 (d + psi - phi),                                         */
/*   d psi/dt = kappa (M_n e - psi),   d phi/dt = kappa M_t e,               */
/* (the n part of the flux is divided by s, the t part multiplied by s).    */
/* The magnetic loss is the matched one on b (damp_b of o_faraday).         */
/* ---------------------------------------------------------------------- */
void o_ampere_pml(const o_mesh *M, const double *b_half, const double *cur, double dt,
                  double mu0, int npml, const int32_t *rows, const double *kappa,
                  const int32_t *n_ptr, const int32_t *n_col, const double *n_val,
                  const int32_t *t_ptr, const int32_t *t_col, const double *t_val,
                  double *psi, double *phi, double *extra, double *d, double *e)
{
    /* d^{n+1} = d^n + dt (C^T [*mu^-1] b^{n+1/2} - i), no loss */
    for (int ed = 0; ed < M->ne; ++ed) {
        if (!M->edge_free[ed]) {
            d[ed] = 0.0;
            continue;
        }
        double curl = 0.0;
        for (int j = 0; j < 2; ++j) {
            int f = M->edge_tri[2 * ed + j];
            if (f < 0) continue;
            curl += M->edge_tsign[2 * ed + j] * (b_half[f] / (mu0 * M->area[f]));
        }
        d[ed] = d[ed] + dt * (curl - cur[ed]);
    }
    /* auxiliary fluxes from e^n (semi-implicit in psi, explicit in phi) */
    for (int k = 0; k < npml; ++k) {
        double x = 0.0, y = 0.0;
        for (int j = n_ptr[k]; j < n_ptr[k + 1]; ++j) x += n_val[j] * e[n_col[j]];
        for (int j = t_ptr[k]; j < t_ptr[k + 1]; ++j) y += t_val[j] * e[t_col[j]];
        double c = kappa[k] * dt;
        psi[k] = (psi[k] * (1.0 - 0.5 * c) + c * x) / (1.0 + 0.5 * c);
        phi[k] = phi[k] + c * y;
        extra[rows[k]] = psi[k] - phi[k];
    }
    /* e^{n+1} = M~ (d^{n+1} + psi - phi) */
    for (int ed = 0; ed < M->ne; ++ed) {
        if (!M->edge_free[ed]) {
            e[ed] = 0.0;
            continue;
        }
        double acc = 0.0;
        for (int j = M->mt_ptr[ed]; j < M->mt_ptr[ed + 1]; ++j)
            acc += M->mt_val[j] * (d[M->mt_col[j]] + extra[M->mt_col[j]]);
        e[ed] = acc;
    }
}
