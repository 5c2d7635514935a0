// Host-side math of the library (compiled with the host compiler, no HIP).
#pragma once

#include <cstdint>
#include <vector>

namespace svh {

// Tucker factors of a real circulant spectrum: Z[kz][ky][kx] =
// sum core[c][b][a] F[0][kx][a] F[1][ky][b] F[2][kz][c].
struct TuckerFactors {
  int d[3] = {0, 0, 0};
  std::vector<double> core;  // [c][b][a], a fastest
  std::vector<double> F[3];  // F[i][k * d[i] + c], k < L[i]
  double relerr = 0;
};

// Face-node topology of the saddle system (eq. 7): incidence matrix A in
// compressed column (one column per basis function a * nvox + k) and
// compressed row (one row per node) form.
struct Topology {
  int M = 0, C = 3, nvox = 0;
  std::vector<int32_t> coords;     // (x, y, z) per voxel
  std::vector<int32_t> face_node;  // node of face 0..5 (-x, +x, -y, +y, -z, +z) per voxel
  std::vector<int> cptr, crow;
  std::vector<double> cval;
  std::vector<int> rptr, rcol;
  std::vector<double> rval;
};
int build_topology(const int K[3], const int32_t* vidx, int nvox, int basis, Topology& t);
void ground_floating(const Topology& t, std::vector<char>& dirichlet);

// Aggregation multigrid of the Schur complement (host setup).
struct AmgLevel {
  int n = 0;
  std::vector<int> rptr, col;
  std::vector<double> val;
};
constexpr int kAmgCoarse = 256;      // stop coarsening at this many nodes
constexpr int kAmgCoarseMax = 1024;  // largest coarsest level inverted densely
constexpr int kAmgMaxLevels = 24;
AmgLevel schur_matrix(const Topology& t, const std::vector<char>& dirichlet, const std::vector<double>& ydiag);
// true if some off-diagonal entry is positive (S is then not an M-matrix: the
// linear basis functions couple opposite faces of a voxel positively)
bool has_positive_coupling(const AmgLevel& A);
// levels[0] = fine; aggs[l][i] = aggregate (node of level l + 1) of node i of
// level l, or -1 for a row without couplings (left out of level l + 1).  Returns how the coarsest level is solved: kAmgCoarseDense
// (coarse_inv = its dense inverse), kAmgCoarseDiagonal (it is diagonal),
// kAmgCoarseJacobi (kAmgCoarseSweeps damped Jacobi sweeps); -1 on failure.
constexpr int kAmgCoarseDense = 0, kAmgCoarseDiagonal = 1, kAmgCoarseJacobi = 2;
constexpr int kAmgCoarseSweeps = 8;
int amg_setup(AmgLevel fine, std::vector<AmgLevel>& levels, std::vector<std::vector<int>>& aggs,
              std::vector<double>& coarse_inv);

// Unit-voxel Green integral T[dz][dy][dx] for offsets 0 <= d < K.
void green_toeplitz_m0(int Kx, int Ky, int Kz, double* T);

// Tucker-SVD (Algorithm 1) of the spectrum of the even circulant embedding of T.
int tucker_even_circulant(const int K[3], const int L[3], const double* T, double tol,
                          TuckerFactors& out);
// Tucker-SVD of the Toeplitz tensor itself (Algorithm 1; Algorithm 2's store):
// factors F[i][k * d_i + c] for k < K[i].  Returns 0, or 1 for a zero tensor.
int tucker_plain(const int K[3], const double* T, double tol, TuckerFactors& out);
// Same for a tensor that is odd along the axes with odd[i] != 0 (sine factors).
// Returns 0, or 1 for a zero tensor (rank-one zero factors).
int tucker_circulant(const int K[3], const int L[3], const double* T, const int odd[3], double tol,
                     TuckerFactors& out);

}  // namespace svh
