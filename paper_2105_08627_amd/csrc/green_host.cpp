// Unit-voxel Green integral (Toeplitz tensor) by closed form, host side.
//
// The voxel-pair integral of eq. 19 / eq. 26 (App. B, dx = 1) for two unit
// cubes whose corners differ by the integer offset d equals the mixed second
// difference, in each axis, of a function F with
//     d^2/dx^2 d^2/dy^2 d^2/dz^2 F(x, y, z) = 1 / sqrt(x^2 + y^2 + z^2):
//     4 pi T(d) = sum_{a,b,c in {-1,0,1}} w_a w_b w_c F(d + (a, b, c)),
// w = (1, -2, 1).  F is the classical Coulomb box-box potential (terms
// x ln(x + r), arctangents and a quartic times r).  The sixth difference
// cancels about |d|^6 of the magnitude of F, so F and the differences are
// evaluated in IEEE binary128 (libquadmath) and rounded to double once.
// F is evaluated once per grid point of [-1, K] per axis and shared by the 27
// stencil terms of every offset.
#include <quadmath.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "host_math.h"

namespace svh {

typedef __float128 qf;

static qf coulomb_F(qf x, qf y, qf z) {
  const qf x2 = x * x, y2 = y * y, z2 = z * z;
  const qf r = sqrtq(x2 + y2 + z2);
  qf s = (x2 * x2 + y2 * y2 + z2 * z2 - 3 * x2 * y2 - 3 * y2 * z2 - 3 * z2 * x2) * r / 60;
  // a * P(b, c) * ln(a + r); P vanishes when b = c = 0, which is also the only
  // case with a + r = 0, so a zero coefficient skips the logarithm.
  const qf cx = (y2 * z2 / 4 - y2 * y2 / 24 - z2 * z2 / 24) * x;
  const qf cy = (x2 * z2 / 4 - x2 * x2 / 24 - z2 * z2 / 24) * y;
  const qf cz = (x2 * y2 / 4 - x2 * x2 / 24 - y2 * y2 / 24) * z;
  if (cx != 0) s += cx * logq(x + r);
  if (cy != 0) s += cy * logq(y + r);
  if (cz != 0) s += cz * logq(z + r);
  // a b c^3 / 6 * atan(a b / (c r)); a zero product means the term vanishes
  const qf kz = x * y * z2 * z / 6;
  const qf ky = x * z * y2 * y / 6;
  const qf kx = y * z * x2 * x / 6;
  if (kz != 0) s -= kz * atanq(x * y / (z * r));
  if (ky != 0) s -= ky * atanq(x * z / (y * r));
  if (kx != 0) s -= kx * atanq(y * z / (x * r));
  return s;
}

// T[(dz*Ky + dy)*Kx + dx], offsets 0 <= d < K, double.
void green_toeplitz_m0(int Kx, int Ky, int Kz, double* T) {
  const int Nx = Kx + 2, Ny = Ky + 2, Nz = Kz + 2;
  std::vector<qf> F((size_t)Nx * Ny * Nz);
#pragma omp parallel for collapse(2) schedule(dynamic, 4)
  for (int k = 0; k < Nz; ++k)
    for (int j = 0; j < Ny; ++j)
      for (int i = 0; i < Nx; ++i)
        F[((size_t)k * Ny + j) * Nx + i] = coulomb_F((qf)(i - 1), (qf)(j - 1), (qf)(k - 1));
  // second difference along x, then y, then z (each shrinks that axis by 2)
  std::vector<qf> Gx((size_t)Kx * Ny * Nz);
#pragma omp parallel for collapse(2)
  for (int k = 0; k < Nz; ++k)
    for (int j = 0; j < Ny; ++j)
      for (int i = 0; i < Kx; ++i) {
        const qf* f = &F[((size_t)k * Ny + j) * Nx + i];
        Gx[((size_t)k * Ny + j) * Kx + i] = f[0] - 2 * f[1] + f[2];
      }
  std::vector<qf>().swap(F);
  std::vector<qf> Gy((size_t)Kx * Ky * Nz);
#pragma omp parallel for collapse(2)
  for (int k = 0; k < Nz; ++k)
    for (int j = 0; j < Ky; ++j)
      for (int i = 0; i < Kx; ++i) {
        const size_t b = ((size_t)k * Ny + j) * Kx + i;
        Gy[((size_t)k * Ky + j) * Kx + i] = Gx[b] - 2 * Gx[b + Kx] + Gx[b + 2 * (size_t)Kx];
      }
  std::vector<qf>().swap(Gx);
  const qf inv4pi = 1 / (4 * M_PIq);
  const size_t plane = (size_t)Kx * Ky;
#pragma omp parallel for collapse(2)
  for (int k = 0; k < Kz; ++k)
    for (int j = 0; j < Ky; ++j)
      for (int i = 0; i < Kx; ++i) {
        const size_t b = ((size_t)k * Ky + j) * Kx + i;
        const qf v = Gy[b] - 2 * Gy[b + plane] + Gy[b + 2 * plane];
        T[b] = (double)(v * inv4pi);
      }
}

}  // namespace svh
