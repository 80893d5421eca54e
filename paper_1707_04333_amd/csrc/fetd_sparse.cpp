// Sparse helpers of the host runtimes (triangles and tetrahedra): the
// Frobenius-norm sparse approximate inverse of a Hodge matrix (Sec. II.A)
// and its residual.
#include "fetd_sparse.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>

namespace fetd {

// Cholesky solve of the small SPD system N x = rhs (n x n, row-major).
bool chol_solve(std::vector<double> &N, int n, std::vector<double> &x)
{
    for (int j = 0; j < n; ++j) {
        double dgn = N[size_t(j) * n + j];
        for (int k = 0; k < j; ++k) dgn -= N[size_t(j) * n + k] * N[size_t(j) * n + k];
        if (!(dgn > 0)) return false;
        dgn = std::sqrt(dgn);
        N[size_t(j) * n + j] = dgn;
        for (int i = j + 1; i < n; ++i) {
            double v = N[size_t(i) * n + j];
            for (int k = 0; k < j; ++k) v -= N[size_t(i) * n + k] * N[size_t(j) * n + k];
            N[size_t(i) * n + j] = v / dgn;
        }
    }
    for (int i = 0; i < n; ++i) {
        double v = x[i];
        for (int k = 0; k < i; ++k) v -= N[size_t(i) * n + k] * x[k];
        x[i] = v / N[size_t(i) * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double v = x[i];
        for (int k = i + 1; k < n; ++k) v -= N[size_t(k) * n + i] * x[k];
        x[i] = v / N[size_t(i) * n + i];
    }
    return true;
}

// Frobenius-norm sparse approximate inverse of [*eps] (Sec. II.A: tunable
// sparsity, exponential convergence in the Frobenius norm): for every free
// column j, minimise ||M m_j - e_j||_2 over m_j supported on the nodes
// within `level` hops of j in the graph of M; solved through the normal
// equations of the small dense block; then symmetrised.
bool spai_build(const Csr &M, const uint8_t *free, int level, Csr &T)
{
    const int ne = int(M.ptr.size()) - 1;
    std::vector<std::vector<int>> pat(ne);
    std::vector<std::vector<double>> sol(ne);
    std::atomic<bool> ok{true};
    const int nthreads = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    auto worker = [&](int t) {
        std::vector<int> mark(ne, -1), rpos(ne, -1);
        std::vector<int> J, I;
        std::vector<double> A, N, x;
        for (int j = t; j < ne; j += nthreads) {
            if (!free[j]) continue;
            J.assign(1, j);
            mark[j] = j;
            size_t head = 0;
            for (int l = 0; l < level; ++l) {
                const size_t end = J.size();
                for (; head < end; ++head)
                    for (int q = M.ptr[J[head]]; q < M.ptr[J[head] + 1]; ++q)
                        if (mark[M.col[q]] != j) {
                            mark[M.col[q]] = j;
                            J.push_back(M.col[q]);
                        }
            }
            std::sort(J.begin(), J.end());
            I.clear();
            for (int cj : J)
                for (int q = M.ptr[cj]; q < M.ptr[cj + 1]; ++q)
                    if (rpos[M.col[q]] != -2 - j) {
                        rpos[M.col[q]] = -2 - j;
                        I.push_back(M.col[q]);
                    }
            std::sort(I.begin(), I.end());
            const int ni = int(I.size()), nj = int(J.size());
            std::vector<int> pos(ni);
            A.assign(size_t(ni) * nj, 0.0);
            // row position lookup by binary search in I
            for (int c = 0; c < nj; ++c) {
                const int cj = J[c];
                for (int q = M.ptr[cj]; q < M.ptr[cj + 1]; ++q) {
                    const int r = int(std::lower_bound(I.begin(), I.end(), M.col[q]) - I.begin());
                    A[size_t(r) * nj + c] = M.val[q];  // M symmetric: column cj = row cj
                }
            }
            N.assign(size_t(nj) * nj, 0.0);
            for (int r = 0; r < ni; ++r)
                for (int p = 0; p < nj; ++p) {
                    const double arp = A[size_t(r) * nj + p];
                    if (arp == 0.0) continue;
                    for (int q = 0; q < nj; ++q) N[size_t(p) * nj + q] += arp * A[size_t(r) * nj + q];
                }
            const int rj = int(std::lower_bound(I.begin(), I.end(), j) - I.begin());
            x.assign(nj, 0.0);
            for (int p = 0; p < nj; ++p) x[p] = A[size_t(rj) * nj + p];
            if (!chol_solve(N, nj, x)) {
                ok = false;
                return;
            }
            pat[j] = J;
            sol[j] = x;
        }
    };
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t) th.emplace_back(worker, t);
    for (auto &x : th) x.join();
    if (!ok) return false;
    // symmetrise: M~_ij = (m_ij + m_ji) / 2 on the symmetric pattern
    T.ptr.assign(ne + 1, 0);
    T.col.clear();
    T.val.clear();
    for (int i = 0; i < ne; ++i) {
        for (size_t a = 0; a < pat[i].size(); ++a) {
            const int j = pat[i][a];
            // value of column j at row i, and of column i at row j
            const double mij = sol[j].empty() ? 0.0 :
                sol[j][std::lower_bound(pat[j].begin(), pat[j].end(), i) - pat[j].begin()];
            const double mji = sol[i][a];
            T.col.push_back(j);
            T.val.push_back(0.5 * (mij + mji));
        }
        T.ptr[i + 1] = int32_t(T.col.size());
    }
    return true;
}

double spai_frobenius(const Csr &M, const Csr &T, const uint8_t *free, int n_free)
{
    // ||I - M M~||_F over the free block, by columns of M~ (symmetric)
    const int ne = int(M.ptr.size()) - 1;
    std::vector<double> acc(ne, 0.0);
    std::vector<int> touched;
    double tot = 0.0;
    for (int j = 0; j < ne; ++j) {
        if (!free[j]) continue;
        touched.clear();
        for (int q = T.ptr[j]; q < T.ptr[j + 1]; ++q) {
            const int k = T.col[q];
            for (int p = M.ptr[k]; p < M.ptr[k + 1]; ++p) {
                if (acc[M.col[p]] == 0.0) touched.push_back(M.col[p]);
                acc[M.col[p]] += M.val[p] * T.val[q];
            }
        }
        bool diag_seen = false;
        for (int r : touched) {
            const double v = acc[r] - (r == j ? 1.0 : 0.0);
            if (r == j) diag_seen = true;
            tot += v * v;
            acc[r] = 0.0;
        }
        if (!diag_seen) tot += 1.0;
    }
    return std::sqrt(tot / std::max(1, n_free));
}

}  // namespace fetd
