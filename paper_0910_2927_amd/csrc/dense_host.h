// Small dense complex FP64 routines on the host (column-major).
#pragma once

#include <complex>
#include <functional>
#include <vector>

namespace sk {
namespace dense {

using cd = std::complex<double>;

void hessenberg(int n, std::vector<cd>& A, std::vector<cd>& Q);
bool schur_hessenberg(int n, std::vector<cd>& H, std::vector<cd>& Q, int max_sweeps);
// A <- T (upper triangular) with A_in = Q T Q^H.
bool schur(int n, std::vector<cd>& A, std::vector<cd>& Q);
// Move the `count` diagonal entries of smallest key to the top, in order.
void reorder_schur(int n, std::vector<cd>& T, std::vector<cd>& Q,
                   const std::function<double(cd)>& key, int count);
bool lu_solve(int n, std::vector<cd> A, std::vector<cd>& B, int r);
bool inverse(int n, const std::vector<cd>& A, std::vector<cd>& X);
bool newton_sign(int n, const std::vector<cd>& A, std::vector<cd>& S, double tol, int maxit);
void matmul(int m, int k, int n, const std::vector<cd>& A, const std::vector<cd>& B,
            std::vector<cd>& C, bool conjA);

}  // namespace dense
}  // namespace sk
