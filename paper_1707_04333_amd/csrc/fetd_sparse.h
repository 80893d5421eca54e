// Sparse helpers shared by the host runtimes.  Not part of the C-ABI.
#pragma once

#include <cstdint>
#include <vector>

namespace fetd {

struct Csr {
    std::vector<int32_t> ptr, col;
    std::vector<double> val;
};

// Cholesky solve of the small SPD system N x = rhs (n x n, row-major; N is
// overwritten).  False if N is not positive definite.
bool chol_solve(std::vector<double> &N, int n, std::vector<double> &x);

// Frobenius-norm sparse approximate inverse of the symmetric matrix M over
// the rows/columns with free[j] != 0: column j minimises ||M m_j - e_j||_2
// over the nodes within `level` hops of j in the graph of M, then the
// result is symmetrised.  False if a normal-equation block is not SPD.
bool spai_build(const Csr &M, const uint8_t *free, int level, Csr &out);

// ||I - M M~||_F over the free block, divided by sqrt(n_free).
double spai_frobenius(const Csr &M, const Csr &T, const uint8_t *free, int n_free);

}  // namespace fetd
