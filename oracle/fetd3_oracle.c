/*
 * FP64 CPU oracle of the FETD-PIC step on tetrahedra (the three-
 * dimensional form of Sec. II: e on edges, b on faces, both Whitney forms
 * evaluated at the particle, the incidence matrices C (faces x edges) and
 * S (cells x faces), the Hodge matrices [*eps] on edges and [*mu^-1] on
 * faces).
 *
 * TEST INFRASTRUCTURE ONLY, like fetd_oracle.c (whose pusher o_push it
 * calls): loaded by the tests, the smoke check and the CPU baseline of the
 * benchmark, never by the HIP library, and sharing no code with it.
 *
 * Conventions (the readings the tests pin):
 *   - tetrahedra are positively oriented; local edges are the pairs
 *     (0,1) (0,2) (0,3) (1,2) (1,3) (2,3), oriented from the lower to the
 *     higher local index; a global edge runs from its lower to its higher
 *     node id and esign = +1 when the two orientations agree;
 *   - local face k is opposite local node k; its Whitney 2-form in local
 *     sorted order (p<q<r) is 2(l_p X_qr + l_q X_rp + l_r X_pq) with
 *     X_ab = grad l_a x grad l_b, whose flux through the face is +1 along
 *     the normal (x_q - x_p) x (x_r - x_p); a global face is the sorted
 *     triple (i<j<l) of node ids with normal (x_j - x_i) x (x_l - x_i) and
 *     fpar = +1 when the local sorted order is an even permutation of it;
 *   - a particle stores its tetrahedron, a derived slot r and the
 *     barycentrics of local nodes (r+1)%4, (r+2)%4, (r+3)%4; the fourth is
 *     ((1 - s0) - s1) - s2;
 *   - the state is d = [*eps] e (FP64), e = M~ d with M~ the approximate
 *     inverse of [*eps]; b holds face fluxes.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

void o_push(int pusher, const double *u, const double *eps, const double *beta,
            double c, double *out);

typedef struct {
    int32_t nt, ne, nf, nn;
    const int32_t *tet_node;   /* [4nt] */
    const int32_t *tet_edge;   /* [6nt] */
    const int8_t *tet_esign;   /* [6nt] */
    const int32_t *tet_face;   /* [4nt] face opposite local node k */
    const int8_t *tet_fpar;    /* [4nt] */
    const int32_t *tet_nbr;    /* [4nt] neighbour across face k, <0 = wall */
    const int8_t *tet_nbrmap;  /* [16nt] for face k: [4k + j] = local index in the
                                  neighbour of local node j (j != k); [4k + k] = the
                                  neighbour's local node opposite the shared face */
    const double *grad;        /* [12nt] grad lambda_k (x, y, z) */
    const double *vxyz;        /* [12nt] image-consistent vertex coordinates */
    const int32_t *face_edge;  /* [3nf] */
    const int8_t *face_esign;  /* [3nf] C entries */
    const uint8_t *edge_free;  /* [ne] */
    const int32_t *mnu_ptr;    /* CSR of [*mu^-1] (faces x faces) */
    const int32_t *mnu_col;
    const double *mnu_val;
    const int32_t *mt_ptr;     /* CSR of M~ (edges x edges) */
    const int32_t *mt_col;
    const double *mt_val;
} o3_mesh;

static const int LE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
static const int LF[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};

static void cross(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

static void local_lambda3(int r, const double *s, double *L)
{
    L[(r + 1) & 3] = s[0];
    L[(r + 2) & 3] = s[1];
    L[(r + 3) & 3] = s[2];
    L[r] = ((1.0 - s[0]) - s[1]) - s[2];
}

/* E = sum over the six local edges of esign e (l_a grad l_b - l_b grad l_a)
   (Sec. II.B with the Whitney 1-forms of a tetrahedron). */
void o3_gather_e(const o3_mesh *M, const double *e, const double *e_ext, int t,
                 const double *L, double *E)
{
    const double *G = M->grad + 12 * t;
    E[0] = E[1] = E[2] = 0.0;
    for (int k = 0; k < 6; ++k) {
        int a = LE[k][0], b = LE[k][1];
        int ed = M->tet_edge[6 * t + k];
        double dof = e[ed];
        if (e_ext) dof = dof + e_ext[ed];
        double s = M->tet_esign[6 * t + k] * dof;
        for (int x = 0; x < 3; ++x)
            E[x] += s * (L[a] * G[3 * b + x] - L[b] * G[3 * a + x]);
    }
}

/* B = sum over the four faces of fpar b_f W2_f (Sec. II.B with the Whitney
   2-forms of a tetrahedron). */
void o3_gather_b(const o3_mesh *M, const double *b, int t, const double *L, double *B)
{
    const double *G = M->grad + 12 * t;
    B[0] = B[1] = B[2] = 0.0;
    for (int k = 0; k < 4; ++k) {
        int p = LF[k][0], q = LF[k][1], r = LF[k][2];
        double Xqr[3], Xrp[3], Xpq[3];
        cross(G + 3 * q, G + 3 * r, Xqr);
        cross(G + 3 * r, G + 3 * p, Xrp);
        cross(G + 3 * p, G + 3 * q, Xpq);
        double s = M->tet_fpar[4 * t + k] * b[M->tet_face[4 * t + k]];
        for (int x = 0; x < 3; ++x)
            B[x] += s * 2.0 * (L[p] * Xqr[x] + L[q] * Xrp[x] + L[r] * Xpq[x]);
    }
}

/* Current of one straight piece inside tetrahedron t from Ls to Lf (Sec.
   II.D, eq. I.assign on the six edges). */
static void deposit3(const o3_mesh *M, int t, const double *Ls, const double *Lf, double qdt,
                     double *cur)
{
    for (int k = 0; k < 6; ++k) {
        int a = LE[k][0], b = LE[k][1];
        double w = Ls[a] * Lf[b] - Lf[a] * Ls[b];
        cur[M->tet_edge[6 * t + k]] += M->tet_esign[6 * t + k] * qdt * w;
    }
}

/*
 * Move by dr, splitting at faces.  Exit rule: with dL_k = grad l_k . dr_rem
 * the candidates are the faces k with dL_k < 0 other than the one just
 * entered, tau_k = max(l_k, 0)/(-dL_k), the smallest wins (ties to the
 * smallest k), tau >= 1 ends inside.  At an exit through face k, with
 * (p, q, w) = (k+1, k+2, k+3) mod 4: l_k = 0, l_p and l_q advance by tau,
 * l_w = (1 - l_p) - l_q; the neighbour inherits them by node identity and
 * its derived slot is the node w.  Returns the number of pieces or -1 when
 * the cap is exceeded; *lost when a wall is met (current deposited up to it).
 */
int o3_move(const o3_mesh *M, int32_t *ptet, int8_t *pslot, double *s3, double dx, double dy,
            double dz, double qdt, double *cur, int cap, int *lost)
{
    int t = *ptet, r = *pslot;
    double L[4], Lf[4];
    local_lambda3(r, s3, L);
    int entry = -1;
    double rx = dx, ry = dy, rz = dz;
    *lost = 0;
    for (int it = 0; it < cap; ++it) {
        const double *G = M->grad + 12 * t;
        double dL[4];
        for (int k = 0; k < 4; ++k) dL[k] = G[3 * k] * rx + G[3 * k + 1] * ry + G[3 * k + 2] * rz;
        int ks = -1;
        double ts = 0.0;
        for (int k = 0; k < 4; ++k) {
            if (k == entry || !(dL[k] < 0.0)) continue;
            double tk = (L[k] > 0.0 ? L[k] : 0.0) / (-dL[k]);
            if (ks < 0 || tk < ts) {
                ks = k;
                ts = tk;
            }
        }
        if (ks < 0 || ts >= 1.0) {
            int a = (r + 1) & 3, b = (r + 2) & 3, c = (r + 3) & 3;
            Lf[a] = L[a] + dL[a];
            Lf[b] = L[b] + dL[b];
            Lf[c] = L[c] + dL[c];
            Lf[r] = ((1.0 - Lf[a]) - Lf[b]) - Lf[c];
            deposit3(M, t, L, Lf, qdt, cur);
            *ptet = t;
            *pslot = (int8_t)r;
            s3[0] = Lf[a];
            s3[1] = Lf[b];
            s3[2] = Lf[c];
            return it + 1;
        }
        int p = (ks + 1) & 3, q = (ks + 2) & 3, w = (ks + 3) & 3;
        Lf[ks] = 0.0;
        Lf[p] = L[p] + ts * dL[p];
        Lf[q] = L[q] + ts * dL[q];
        Lf[w] = (1.0 - Lf[p]) - Lf[q];
        deposit3(M, t, L, Lf, qdt, cur);
        int nb = M->tet_nbr[4 * t + ks];
        if (nb < 0) {
            *lost = 1;
            *ptet = t;
            *pslot = (int8_t)w;
            s3[0] = Lf[(w + 1) & 3];
            s3[1] = Lf[(w + 2) & 3];
            s3[2] = Lf[(w + 3) & 3];
            return it + 1;
        }
        const int8_t *mp = M->tet_nbrmap + 16 * t + 4 * ks;
        double Ln[4];
        Ln[mp[ks]] = 0.0;
        Ln[mp[p]] = Lf[p];
        Ln[mp[q]] = Lf[q];
        Ln[mp[w]] = Lf[w];
        memcpy(L, Ln, sizeof L);
        r = mp[w];
        entry = mp[ks];
        t = nb;
        double sc = 1.0 - ts;
        rx = rx * sc;
        ry = ry * sc;
        rz = rz * sc;
    }
    return -1;
}

/* b^{n+1/2} = b^{n-1/2} - dt C e^n (Sec. II.A, eq. semi.dis.curl.1). */
void o3_faraday(const o3_mesh *M, const double *b_old, const double *e, double dt,
                double *b_new)
{
    for (int f = 0; f < M->nf; ++f) {
        double circ = 0.0;
        for (int k = 0; k < 3; ++k)
            circ += M->face_esign[3 * f + k] * e[M->face_edge[3 * f + k]];
        b_new[f] = b_old[f] - dt * circ;
    }
}

/*
 * d^{n+1} = d^n + dt (C^T [*mu^-1] b^{n+1/2} - i^{n+1/2}) on free edges,
 * e^{n+1} = M~ d^{n+1} (Sec. II.A, eq. semi.dis.curl.2 in the d form).
 * h = [*mu^-1] b is one sparse product; C^T h is accumulated face by face
 * in increasing face order.  work holds nf + ne doubles.
 */
void o3_ampere(const o3_mesh *M, const double *b_half, const double *cur, double dt, double *d,
               double *e, double *work)
{
    double *h = work, *t = work + M->nf;
    for (int f = 0; f < M->nf; ++f) {
        double acc = 0.0;
        for (int j = M->mnu_ptr[f]; j < M->mnu_ptr[f + 1]; ++j)
            acc += M->mnu_val[j] * b_half[M->mnu_col[j]];
        h[f] = acc;
    }
    for (int ed = 0; ed < M->ne; ++ed) t[ed] = 0.0;
    for (int f = 0; f < M->nf; ++f)
        for (int k = 0; k < 3; ++k) {
            int ed = M->face_edge[3 * f + k];
            t[ed] = t[ed] + M->face_esign[3 * f + k] * h[f];
        }
    for (int ed = 0; ed < M->ne; ++ed)
        d[ed] = M->edge_free[ed] ? d[ed] + dt * (t[ed] - cur[ed]) : 0.0;
    for (int ed = 0; ed < M->ne; ++ed) {
        if (!M->edge_free[ed]) {
            e[ed] = 0.0;
            continue;
        }
        double acc = 0.0;
        for (int j = M->mt_ptr[ed]; j < M->mt_ptr[ed + 1]; ++j) acc += M->mt_val[j] * d[M->mt_col[j]];
        e[ed] = acc;
    }
}

/*
 * Particle stage of one species: gather E^n and B^n = (B^{n+1/2} +
 * B^{n-1/2})/2 (plus b_ext [3nt] per tetrahedron, optional), push, move,
 * deposit.  Returns 0, -1 (crossing cap) or -2 (non-finite momentum) with
 * *bad the first offending particle; counts[0] += pieces, counts[1] += lost.
 */
int o3_particles(const o3_mesh *M, const double *e, const double *e_ext, const double *b_old,
                 const double *b_new, const double *b_ext, int pusher, double q, double m,
                 double w, double dt, double c, int cap, int64_t n, int32_t *tet, int8_t *slot,
                 double *lam, double *u, double *cur, double *bavg, int64_t *counts, int64_t *bad)
{
    double alpha = q * dt / (2.0 * m);
    double qdt = q * w / dt;
    for (int f = 0; f < M->nf; ++f) bavg[f] = 0.5 * (b_new[f] + b_old[f]);
    for (int64_t p = 0; p < n; ++p) {
        int t = tet[p];
        if (t < 0) continue;
        double L[4], E[3], B[3];
        local_lambda3(slot[p], lam + 3 * p, L);
        o3_gather_e(M, e, e_ext, t, L, E);
        o3_gather_b(M, bavg, t, L, B);
        if (b_ext)
            for (int x = 0; x < 3; ++x) B[x] += b_ext[3 * t + x];
        double eps[3], beta[3], u1[3];
        for (int x = 0; x < 3; ++x) {
            eps[x] = alpha * E[x];
            beta[x] = alpha * B[x];
        }
        o_push(pusher, u + 3 * p, eps, beta, c, u1);
        if (!isfinite(u1[0]) || !isfinite(u1[1]) || !isfinite(u1[2])) {
            *bad = p;
            return -2;
        }
        memcpy(u + 3 * p, u1, sizeof u1);
        double g = sqrt(1.0 + (u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]) / (c * c));
        int32_t t32 = t;
        int8_t s8 = slot[p];
        int lost = 0;
        int ns = o3_move(M, &t32, &s8, lam + 3 * p, dt * u1[0] / g, dt * u1[1] / g, dt * u1[2] / g,
                         qdt, cur, cap, &lost);
        if (ns < 0) {
            *bad = p;
            return -1;
        }
        counts[0] += ns;
        if (lost) counts[1] += 1;
        tet[p] = lost ? -1 : t32;
        slot[p] = s8;
    }
    return 0;
}

/* Nodal charge q_i = sum_p Q lambda_i(r_p) (Sec. II.D). */
void o3_charge(const o3_mesh *M, double qw, int64_t n, const int32_t *tet, const int8_t *slot,
               const double *lam, double *qn)
{
    for (int64_t p = 0; p < n; ++p) {
        int t = tet[p];
        if (t < 0) continue;
        double L[4];
        local_lambda3(slot[p], lam + 3 * p, L);
        for (int k = 0; k < 4; ++k) qn[M->tet_node[4 * t + k]] += qw * L[k];
    }
}
