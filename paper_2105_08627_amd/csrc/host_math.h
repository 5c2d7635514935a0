// Host-side math of the library (compiled with the host compiler, no HIP).
#pragma once

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

// Unit-voxel Green integral T[dz][dy][dx] for offsets 0 <= d < K.
void green_toeplitz_m0(int Kx, int Ky, int Kz, double* T);

// Tucker-SVD (Algorithm 1) of the spectrum of the even circulant embedding of T.
int tucker_even_circulant(const int K[3], const int L[3], const double* T, double tol,
                          TuckerFactors& out);

}  // namespace svh
