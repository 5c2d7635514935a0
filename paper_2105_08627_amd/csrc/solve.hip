// Port solve of the saddle system (eq. 7) on the device, FP64.
//
//   K [I; Phi_F] = [A_D^T Phi_D; 0],  K = [[Z, -A_F^T], [A_F, 0]]
//
// Right-preconditioned flexible GMRES (restart m, Sec. III settings), all
// port excitations in lockstep.  The preconditioner is the sparse saddle
// matrix of eq. 12 with Y = |diag Z|, applied through its Schur complement
// (eqs. 13-15): e = d - A Y^-1 c, S b = e with S = A Y^-1 A^T (real, SPD on
// the free nodes), a = Y^-1 (c + A^T b).  S b = e is solved by Jacobi-
// preconditioned conjugate gradients on the device; since that inner solve
// is inexact the outer method is the flexible variant.  Gram-Schmidt runs
// twice (CGS2) with all inner products in FP64 on the device; only the
// Hessenberg column (a few scalars per port) crosses to the host per step.
//
// Vector layout: per port one column of N = C*K + M complex doubles,
// currents (component-major, as for svh_matvec) then one potential per node.
// Dirichlet (port and grounded) node entries are kept at zero.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>

#include "host_math.h"
#include "svh_internal.h"

namespace svh {

typedef std::complex<double> cd;

__device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 zsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zcmul(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 zscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

#define GRID_STRIDE(i, n) \
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long long)gridDim.x * blockDim.x)

// ------------------------------------------------------------- operator --
// After y_I = Z x_I: y_I -= A^T x_Phi and y_Phi = A x_I on free nodes
// (transpose: y_I += A^T x_Phi, y_Phi = -A x_I).
__global__ void k_saddle_fix(int nrhs, long long N, int CK, int M, const int* __restrict__ cptr,
                             const int* __restrict__ crow, const double* __restrict__ cval,
                             const int* __restrict__ rptr, const int* __restrict__ rcol,
                             const double* __restrict__ rval, const uint8_t* __restrict__ freem,
                             const double2* __restrict__ x, double2* __restrict__ y, int transpose) {
  const long long per = (long long)CK + M;
  GRID_STRIDE(i, per * nrhs) {
    const long long r = i / per, idx = i % per;
    const double2* xr = x + r * N;
    double2* yr = y + r * N;
    if (idx < CK) {
      double2 acc = make_double2(0, 0);
      for (int q = cptr[idx]; q < cptr[idx + 1]; ++q) acc = zadd(acc, zscale(xr[CK + crow[q]], cval[q]));
      yr[idx] = transpose ? zadd(yr[idx], acc) : zsub(yr[idx], acc);
    } else {
      const int m = (int)(idx - CK);
      double2 acc = make_double2(0, 0);
      if (freem[m])
        for (int q = rptr[m]; q < rptr[m + 1]; ++q) acc = zadd(acc, zscale(xr[rcol[q]], rval[q]));
      yr[idx] = transpose ? zscale(acc, -1.0) : acc;
    }
  }
}

// ------------------------------------------------------- preconditioner --
// e = d - A Y^-1 c (free rows; transpose: d + A Y^-1 c), into node vector e
__global__ void k_pre_rhs(int nrhs, long long N, int CK, int M, const int* __restrict__ rptr,
                          const int* __restrict__ rcol, const double* __restrict__ rval,
                          const uint8_t* __restrict__ freem, const double* __restrict__ ydiag,
                          const double2* __restrict__ in, double2* __restrict__ e, int transpose) {
  GRID_STRIDE(i, (long long)M * nrhs) {
    const long long r = i / M;
    const int m = (int)(i % M);
    const double2* c = in + r * N;
    double2 acc = make_double2(0, 0);
    if (freem[m]) {
      for (int q = rptr[m]; q < rptr[m + 1]; ++q) acc = zadd(acc, zscale(c[rcol[q]], rval[q] / ydiag[rcol[q]]));
      const double2 d = c[CK + m];
      acc = transpose ? zadd(d, acc) : zsub(d, acc);
    }
    e[r * M + m] = acc;
  }
}

// The sparse products of the Schur solve take one row for up to kRowRhs
// right-hand sides per thread: the row's entries are read once and the
// gathers of the right-hand sides are independent (a missing right-hand
// side's index is clamped to the last one, so every load is unconditional;
// only the stores are masked).  Each element sums in the row's order.
constexpr int kRowRhs = 8;

// acc[j] += sgn * sum_q a[q] * x[off[j] + c[q]] over q in [q0, q1), four
// entries at a time so that their index loads and gathers are in flight
// together (the additions keep the entry order)
template <int SGN>
__device__ __forceinline__ void row_gather(int q0, int q1, const int* __restrict__ c, const double* __restrict__ a,
                                           const double2* __restrict__ x, const long long* off, double2* acc) {
  int q = q0;
  for (; q + 4 <= q1; q += 4) {
    const int c0 = c[q], c1 = c[q + 1], c2 = c[q + 2], c3 = c[q + 3];
    const double a0 = SGN * a[q], a1 = SGN * a[q + 1], a2 = SGN * a[q + 2], a3 = SGN * a[q + 3];
#pragma unroll
    for (int j = 0; j < kRowRhs; ++j) {
      const double2 x0 = x[off[j] + c0], x1 = x[off[j] + c1], x2 = x[off[j] + c2], x3 = x[off[j] + c3];
      acc[j] = zadd(acc[j], zscale(x0, a0));
      acc[j] = zadd(acc[j], zscale(x1, a1));
      acc[j] = zadd(acc[j], zscale(x2, a2));
      acc[j] = zadd(acc[j], zscale(x3, a3));
    }
  }
  for (; q < q1; ++q) {
    const int cq = c[q];
    const double aq = SGN * a[q];
#pragma unroll
    for (int j = 0; j < kRowRhs; ++j) acc[j] = zadd(acc[j], zscale(x[off[j] + cq], aq));
  }
}

// u = Y^-1 A^T v (basis-sized), v a node vector with zero Dirichlet entries
__global__ void k_s_half(int nrhs, int CK, int M, const int* __restrict__ cptr, const int* __restrict__ crow,
                         const double* __restrict__ cval, const double* __restrict__ ydiag,
                         const double2* __restrict__ v, double2* __restrict__ u) {
  const int nchunk = (nrhs + kRowRhs - 1) / kRowRhs;
  GRID_STRIDE(i, (long long)CK * nchunk) {
    const int b = (int)(i % CK);
    const int r0 = (int)(i / CK) * kRowRhs;
    const int last = nrhs - 1 - r0;  // >= 0
    long long off[kRowRhs];
    double2 acc[kRowRhs];
#pragma unroll
    for (int j = 0; j < kRowRhs; ++j) {
      off[j] = (long long)(r0 + min(j, last)) * M;
      acc[j] = make_double2(0, 0);
    }
    row_gather<1>(cptr[b], cptr[b + 1], crow, cval, v, off, acc);
    const double yi = 1.0 / ydiag[b];
#pragma unroll
    for (int j = 0; j < kRowRhs; ++j)
      if (j <= last) u[(long long)(r0 + j) * CK + b] = zscale(acc[j], yi);
  }
}

// q = A u on free nodes (S v = A Y^-1 A^T v)
__global__ void k_s_full(int nrhs, int CK, int M, const int* __restrict__ rptr, const int* __restrict__ rcol,
                         const double* __restrict__ rval, const uint8_t* __restrict__ freem,
                         const double2* __restrict__ u, double2* __restrict__ q) {
  const int nchunk = (nrhs + kRowRhs - 1) / kRowRhs;
  GRID_STRIDE(i, (long long)M * nchunk) {
    const int m = (int)(i % M);
    const int r0 = (int)(i / M) * kRowRhs;
    const int last = nrhs - 1 - r0;  // >= 0
    long long off[kRowRhs];
    double2 acc[kRowRhs];
#pragma unroll
    for (int j = 0; j < kRowRhs; ++j) {
      off[j] = (long long)(r0 + min(j, last)) * CK;
      acc[j] = make_double2(0, 0);
    }
    if (freem[m]) row_gather<1>(rptr[m], rptr[m + 1], rcol, rval, u, off, acc);
#pragma unroll
    for (int j = 0; j < kRowRhs; ++j)
      if (j <= last) q[(long long)(r0 + j) * M + m] = acc[j];
  }
}

// a = Y^-1 (c + A^T b) (transpose: Y^-1 (c - A^T b)); out = [a; b]
__global__ void k_pre_out(int nrhs, long long N, int CK, int M, const int* __restrict__ cptr,
                          const int* __restrict__ crow, const double* __restrict__ cval,
                          const double* __restrict__ ydiag, const double2* __restrict__ in,
                          const double2* __restrict__ bsol, double2* __restrict__ out, int transpose) {
  const long long per = (long long)CK + M;
  GRID_STRIDE(i, per * nrhs) {
    const long long r = i / per, idx = i % per;
    const double2* br = bsol + r * M;
    if (idx < CK) {
      double2 acc = make_double2(0, 0);
      for (int q = cptr[idx]; q < cptr[idx + 1]; ++q) acc = zadd(acc, zscale(br[crow[q]], cval[q]));
      const double2 c = in[r * N + idx];
      out[r * N + idx] = zscale(transpose ? zsub(c, acc) : zadd(c, acc), 1.0 / ydiag[idx]);
    } else {
      out[r * N + idx] = br[idx - CK];
    }
  }
}

// ------------------------------------------------------------ reductions --
// part[g][blk] = sum over the block's chunk of conj(X_g) * Y_g, where pair g
// = (i, r) reads X at X + i * xs_i + r * xs_r and Y at Y + r * ys_r.
__global__ void __launch_bounds__(256) k_mdot(long long n, int nrhs, const double2* __restrict__ X, long long xs_i,
                                              long long xs_r, const double2* __restrict__ Y, long long ys_r,
                                              double2* __restrict__ part, int conj_x) {
  __shared__ double2 sh[256];
  const int g = blockIdx.y;
  const int i = g / nrhs, r = g % nrhs;
  const double2* xp = X + (long long)i * xs_i + (long long)r * xs_r;
  const double2* yp = Y + (long long)r * ys_r;
  double2 acc = make_double2(0, 0);
  for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < n; k += (long long)gridDim.x * 256)
    acc = zadd(acc, conj_x ? zcmul(xp[k], yp[k]) : zmul(xp[k], yp[k]));
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = zadd(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long long)g * gridDim.x + blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256) k_psum(int nb, const double2* __restrict__ part, double2* __restrict__ out) {
  __shared__ double2 sh[256];
  const int g = blockIdx.x;
  double2 acc = make_double2(0, 0);
  for (int k = threadIdx.x; k < nb; k += 256) acc = zadd(acc, part[(long long)g * nb + k]);
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = zadd(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[g] = sh[0];
}

// ------------------------------------------------------------------ PCG --
// r = e, b = 0, z = D^-1 r, p = z
__global__ void k_pcg_init(long long n, int M, const double* __restrict__ sdiag, const uint8_t* __restrict__ freem,
                           const double2* __restrict__ e, double2* __restrict__ r, double2* __restrict__ z,
                           double2* __restrict__ p, double2* __restrict__ b) {
  GRID_STRIDE(i, n) {
    const int m = (int)(i % M);
    const double2 v = e[i];
    r[i] = v;
    const double2 zz = freem[m] ? zscale(v, 1.0 / sdiag[m]) : make_double2(0, 0);
    z[i] = zz;
    p[i] = zz;
    b[i] = make_double2(0, 0);
  }
}

// alpha = rho / Re(p^H q) per right-hand side (0 when converged or degenerate)
__global__ void k_pcg_alpha(int nrhs, const double2* __restrict__ rho, const double2* __restrict__ pq,
                            double* __restrict__ alpha) {
  const int r = threadIdx.x;
  if (r < nrhs) alpha[r] = (pq[r].x > 0 && rho[r].x > 0) ? rho[r].x / pq[r].x : 0.0;
}

// b += alpha p, r -= alpha q, z = D^-1 r
__global__ void k_pcg_update(long long n, int M, const double* __restrict__ sdiag, const uint8_t* __restrict__ freem,
                             const double* __restrict__ alpha, const double2* __restrict__ p,
                             const double2* __restrict__ q, double2* __restrict__ b, double2* __restrict__ r,
                             double2* __restrict__ z) {
  GRID_STRIDE(i, n) {
    const int m = (int)(i % M);
    const double a = alpha[i / M];
    b[i] = zadd(b[i], zscale(p[i], a));
    const double2 rr = zsub(r[i], zscale(q[i], a));
    r[i] = rr;
    z[i] = freem[m] ? zscale(rr, 1.0 / sdiag[m]) : make_double2(0, 0);
  }
}

// beta = rho_new / rho; rho = rho_new
__global__ void k_pcg_beta(int nrhs, double2* __restrict__ rho, const double2* __restrict__ rho_new,
                           double* __restrict__ beta) {
  const int r = threadIdx.x;
  if (r < nrhs) {
    beta[r] = rho[r].x > 0 ? rho_new[r].x / rho[r].x : 0.0;
    rho[r] = rho_new[r];
  }
}

__global__ void k_pcg_dir(long long n, int M, const double* __restrict__ beta, const double2* __restrict__ z,
                          double2* __restrict__ p) {
  GRID_STRIDE(i, n) p[i] = zadd(z[i], zscale(p[i], beta[i / M]));
}

// ------------------------------------------------ multigrid V-cycle (S) --
// Batched over right-hand sides: vectors [r][n] of complex values, level
// matrices real CSR.  wdinv = w_i / a_ii with the Jacobi weight w_i = 0.7, or
// 1 on rows without couplings (solved exactly); the coarse correction is
// scaled by kAmgAlpha < 2 (plain aggregation under-corrects), which keeps the
// cycle symmetric positive definite.
constexpr double kAmgOmega = 0.7;
constexpr double kAmgAlpha = 1.8;

__global__ void k_amg_smooth0(int nrhs, int n, const double* __restrict__ wdinv, const double2* __restrict__ b,
                              double2* __restrict__ x) {
  GRID_STRIDE(i, (long long)n * nrhs) x[i] = zscale(b[i], wdinv[i % n]);
}
// r = b - A x, one row for up to kRowRhs right-hand sides per thread.
__global__ void k_amg_resid(int nrhs, int n, const int* __restrict__ rptr, const int* __restrict__ col,
                            const double* __restrict__ val, const double2* __restrict__ b,
                            const double2* __restrict__ x, double2* __restrict__ r) {
  const int nchunk = (nrhs + kRowRhs - 1) / kRowRhs;
  GRID_STRIDE(i, (long long)n * nchunk) {
    const int row = (int)(i % n);
    const int r0 = (int)(i / n) * kRowRhs;
    const int last = nrhs - 1 - r0;  // >= 0
    long long off[kRowRhs];
    double2 acc[kRowRhs];
#pragma unroll
    for (int j = 0; j < kRowRhs; ++j) {
      off[j] = (long long)(r0 + min(j, last)) * n;
      acc[j] = b[off[j] + row];
    }
    row_gather<-1>(rptr[row], rptr[row + 1], col, val, x, off, acc);
#pragma unroll
    for (int j = 0; j < kRowRhs; ++j)
      if (j <= last) r[off[j] + row] = acc[j];
  }
}
// r = b - A x on a small level, whose few rows leave most of the chip idle
// with one thread per row: one wavefront per row instead.  Lane t takes
// right-hand side t % 16 of the current group of 16 and the row's entries
// t / 16, t / 16 + 4, ...; the four partial sums meet through lane exchanges.
__global__ void k_amg_resid_w(int nrhs, int n, const int* __restrict__ rptr, const int* __restrict__ col,
                              const double* __restrict__ val, const double2* __restrict__ b,
                              const double2* __restrict__ x, double2* __restrict__ r) {
  const int lane = threadIdx.x & 63, rl = lane & 15, g = lane >> 4;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long row = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6; row < n; row += nwaves) {
    const int q0 = rptr[row], q1 = rptr[row + 1];
    for (int r0 = 0; r0 < nrhs; r0 += 16) {
      const long long off = (long long)min(r0 + rl, nrhs - 1) * n;
      double2 acc = make_double2(0, 0);
      for (int q = q0 + g; q < q1; q += 4) acc = zadd(acc, zscale(x[off + col[q]], val[q]));
      acc.x += __shfl_xor(acc.x, 16);
      acc.y += __shfl_xor(acc.y, 16);
      acc.x += __shfl_xor(acc.x, 32);
      acc.y += __shfl_xor(acc.y, 32);
      if (g == 0 && r0 + rl < nrhs) r[off + row] = zsub(b[off + row], acc);
    }
  }
}
constexpr int kWaveRowLevel = 32768;  // levels with fewer rows take a wavefront per row

__global__ void k_amg_jacobi(int nrhs, int n, const double* __restrict__ wdinv, const double2* __restrict__ r,
                             double2* __restrict__ x) {
  GRID_STRIDE(i, (long long)n * nrhs) x[i] = zadd(x[i], zscale(r[i], wdinv[i % n]));
}
// bc[I] = sum of r over the members of aggregate I
__global__ void k_amg_restrict(int nrhs, int nf, int nc, const int* __restrict__ mptr, const int* __restrict__ mem,
                               const double2* __restrict__ r, double2* __restrict__ bc) {
  GRID_STRIDE(i, (long long)nc * nrhs) {
    const long long rf = (i / nc) * nf;
    const int I = (int)(i % nc);
    double2 acc = make_double2(0, 0);
    for (int k = mptr[I]; k < mptr[I + 1]; ++k) acc = zadd(acc, r[rf + mem[k]]);
    bc[i] = acc;
  }
}
// x += alpha P xc (rows left out of the coarse level have agg < 0)
__global__ void k_amg_prolong(int nrhs, int nf, int nc, const int* __restrict__ agg, const double2* __restrict__ xc,
                              double2* __restrict__ x) {
  GRID_STRIDE(i, (long long)nf * nrhs) {
    const int a = agg[i % nf];
    if (a >= 0) x[i] = zadd(x[i], zscale(xc[(i / nf) * nc + a], kAmgAlpha));
  }
}
// x = Cinv b on the coarsest level (dense, row-major)
__global__ void k_amg_coarse(int nrhs, int n, const double* __restrict__ cinv, const double2* __restrict__ b,
                             double2* __restrict__ x) {
  GRID_STRIDE(i, (long long)n * nrhs) {
    const long long base = (i / n) * n;
    const double* row = cinv + (long long)(i % n) * n;
    double2 acc = make_double2(0, 0);
    for (int j = 0; j < n; ++j) acc = zadd(acc, zscale(b[base + j], row[j]));
    x[i] = acc;
  }
}

// ---------------------------------------------------------------- GMRES --
// w -= sum_{i<=j} h[i][r] V_i  (h on the device, from k_mdot/k_psum)
__global__ void k_cgs_update(long long N, int nrhs, int ni, const double2* __restrict__ V, long long vs_i,
                             const double2* __restrict__ h, double2* __restrict__ w) {
  GRID_STRIDE(k, N * nrhs) {
    const long long r = k / N, n = k % N;
    double2 acc = w[k];
    for (int i = 0; i < ni; ++i) acc = zsub(acc, zmul(h[i * nrhs + r], V[(long long)i * vs_i + r * N + n]));
    w[k] = acc;
  }
}

// hh[i][r] += h2[i][r]
__global__ void k_add_small(int n, double2* __restrict__ a, const double2* __restrict__ b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = zadd(a[i], b[i]);
}

// V[r] = w[r] / sqrt(nrm2[r]) (0 if the norm vanishes)
__global__ void k_normalize(long long N, int nrhs, const double2* __restrict__ nrm2, const double2* __restrict__ w,
                            double2* __restrict__ v) {
  GRID_STRIDE(k, N * nrhs) {
    const double s = nrm2[k / N].x;
    v[k] = s > 0 ? zscale(w[k], 1.0 / sqrt(s)) : make_double2(0, 0);
  }
}

// x[r] += sum_j coef[j][r] Z_j[r]
__global__ void k_combine(long long N, int nrhs, int nj, const double2* __restrict__ Zk, long long zs_j,
                          const double2* __restrict__ coef, double2* __restrict__ x) {
  GRID_STRIDE(k, N * nrhs) {
    const long long r = k / N, n = k % N;
    double2 acc = x[k];
    for (int j = 0; j < nj; ++j) acc = zadd(acc, zmul(coef[j * nrhs + r], Zk[(long long)j * zs_j + r * N + n]));
    x[k] = acc;
  }
}

// out = b - out (residual from out = K x)
__global__ void k_resid(long long n, const double2* __restrict__ b, double2* __restrict__ out) {
  GRID_STRIDE(i, n) out[i] = zsub(b[i], out[i]);
}

// rhs[r] = [b_r (real port vector); 0]
__global__ void k_port_rhs(int nrhs, long long N, int CK, const double* __restrict__ bport,
                           double2* __restrict__ rhs) {
  GRID_STRIDE(k, N * nrhs) {
    const long long r = k / N, n = k % N;
    rhs[k] = n < CK ? make_double2(bport[r * CK + n], 0.0) : make_double2(0, 0);
  }
}

__global__ void k_add(long long n, const double2* __restrict__ a, double2* __restrict__ b) {
  GRID_STRIDE(i, n) b[i] = zadd(b[i], a[i]);
}
__global__ void k_copy(long long n, const double2* __restrict__ a, double2* __restrict__ b) {
  GRID_STRIDE(i, n) b[i] = a[i];
}
__global__ void k_zero(long long n, double2* __restrict__ a) {
  GRID_STRIDE(i, n) a[i] = make_double2(0, 0);
}

// Derivative of the admittance with respect to p_k = lambda_k^-2 (London
// depth): only the voxel self terms m_beta c_k / dx of Z depend on p_k
// (m_beta = 1 for the constant basis functions, 1/6 and 1/2 for the linear
// ones), with dc/dp = j c^2 / (w mu0) (from eq. 3, c = 1/sigma).  With the
// adjoint solutions y_q of K^T y_q = [b_q; 0],
//   dY[q][p][k] = - sum_beta m_beta y_q[beta, k] x_p[beta, k] * j c_k^2 / (w mu0 dx).
__global__ void k_port_grad(int nports, int C, int K, long long N, const double2* __restrict__ cdiag,
                            double inv_wmu, const double2* __restrict__ xf, const double2* __restrict__ xa,
                            double2* __restrict__ dY) {
  GRID_STRIDE(i, (long long)K * nports * nports) {
    const int k = (int)(i % K);
    const long long qp = i / K;
    const int q = (int)(qp / nports), pp = (int)(qp % nports);
    double2 acc = make_double2(0, 0);
    for (int b = 0; b < C; ++b) {
      const double m = b < 3 ? 1.0 : b == 3 ? 1.0 / 6.0 : 0.5;
      const double2 t = zmul(xa[q * N + (long long)b * K + k], xf[pp * N + (long long)b * K + k]);
      acc = zadd(acc, make_double2(m * t.x, m * t.y));
    }
    // cdiag holds c / dx; dz/dp = j c^2 / (w mu0 dx) = j (c/dx)^2 dx / (w mu0)
    const double2 cd = cdiag[k];
    const double2 c2 = zmul(cd, cd);
    const double2 dz = make_double2(-c2.y * inv_wmu, c2.x * inv_wmu);
    const double2 t = zmul(acc, dz);
    dY[i] = make_double2(-t.x, -t.y);
  }
}

// grad[k] = Im( sum_{q,p} W[q][p] dY[q][p][k] ) * scale
__global__ void k_grad_contract(int nports, int K, const double2* __restrict__ W, const double2* __restrict__ dY,
                                double scale, double* __restrict__ grad) {
  GRID_STRIDE(k, (long long)K) {
    double acc = 0;
    for (int g = 0; g < nports * nports; ++g) {
      const double2 a = W[g], b = dY[(long long)g * K + k];
      acc += a.x * b.y + a.y * b.x;
    }
    grad[k] = acc * scale;
  }
}

// Y[q][p] = b_q^T I_p (no conjugation), partial sums per block
__global__ void __launch_bounds__(256) k_ydot(int CK, int nports, long long N, const double* __restrict__ bport,
                                              const double2* __restrict__ X, double2* __restrict__ part) {
  __shared__ double2 sh[256];
  const int g = blockIdx.y;
  const int q = g / nports, pp = g % nports;
  double2 acc = make_double2(0, 0);
  for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < CK; k += (long long)gridDim.x * 256)
    acc = zadd(acc, zscale(X[pp * N + k], bport[(long long)q * CK + k]));
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = zadd(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long long)g * gridDim.x + blockIdx.x] = sh[0];
}

}  // namespace svh

// ======================================================================
// host side
// ======================================================================
namespace svh {

namespace {

// Progress lines of the solver on stderr (svh_problem::verbose, or the
// SVH_VERBOSE environment variable at the first solve).
bool verbose(svh_problem* p) {
  if (p->verbose < 0) {
    const char* e = std::getenv("SVH_VERBOSE");
    p->verbose = (e && *e && *e != '0') ? 1 : 0;
  }
  return p->verbose > 0;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

svh_status sfail(svh_problem* p, svh_status st, const std::string& m) {
  p->err = m;
  return st;
}

#define SCHK(call)                                                                         \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return sfail(p, e_ == hipErrorOutOfMemory ? SVH_ENOMEM : SVH_EHIP,                   \
                   std::string(#call) + ": " + hipGetErrorString(e_));                     \
  } while (0)

template <typename T>
hipError_t up(T** dst, const T* src, size_t n) {
  if (*dst) (void)hipFree(*dst);
  *dst = nullptr;
  if (n == 0) return hipSuccess;
  hipError_t e = hipMalloc(dst, n * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
}

template <typename T>
void fr(T*& ptr) {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
}

int nblocks(long long n) {
  long long b = (n + 255) / 256;
  return (int)std::max(1LL, std::min(b, 8192LL));
}
// grid of the row kernels: one thread per row and group of kRowRhs right-hand sides
int resid_blocks(int n, int nrhs) { return nblocks((long long)n * ((nrhs + kRowRhs - 1) / kRowRhs)); }

// r = b - A x on one multigrid level (wavefront per row on small levels)
void amg_resid(const svh_problem::AmgDev& L, int nr, const double2* b, const double2* x, double2* r, hipStream_t s) {
  if (L.n < kWaveRowLevel)
    hipLaunchKernelGGL(k_amg_resid_w, dim3(nblocks(64LL * L.n)), dim3(256), 0, s, nr, L.n, L.rptr, L.col, L.val, b, x,
                       r);
  else
    hipLaunchKernelGGL(k_amg_resid, dim3(resid_blocks(L.n, nr)), dim3(256), 0, s, nr, L.n, L.rptr, L.col, L.val, b, x,
                       r);
}

constexpr int kDotBlocks = 256;

struct SolveWs {
  double2 *V, *Zk, *W, *Rhs, *E, *R, *Zp, *P, *Q, *Bs, *U, *part, *h, *h2, *nrm, *rho, *rhon, *pq, *D, *Rr;
  float2 *x32, *y32;
  double *alpha, *beta;
  void *mv, *mv32;
  size_t mv_bytes, mv32_bytes;
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Carves the caller's workspace; returns the bytes needed (ws may be null).
size_t carve(const svh_problem* p, int restart, svh_prec prec, char* ws, SolveWs* w) {
  const long long CK = (long long)p->C * p->nvox, M = p->topo.M, N = CK + M;
  const int nr = std::max(1, p->nports);
  const bool ir = prec == SVH_FP32_IR;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* q = ws ? ws + off : nullptr;
    off += align256(bytes);
    return q;
  };
  const size_t z = sizeof(double2);
  char* V = take((size_t)(restart + 1) * nr * N * z);
  char* Zk = take((size_t)restart * nr * N * z);
  char* W = take((size_t)nr * N * z);
  char* Rhs = take((size_t)nr * N * z);
  char* E = take((size_t)nr * M * z);
  char* R = take((size_t)nr * M * z);
  char* Zp = take((size_t)nr * M * z);
  char* P = take((size_t)nr * M * z);
  char* Q = take((size_t)nr * M * z);
  char* Bs = take((size_t)nr * M * z);
  char* U = take((size_t)nr * CK * z);
  char* part = take((size_t)kDotBlocks * (restart + 1) * nr * z);
  char* h = take((size_t)(restart + 2) * nr * z);
  char* h2 = take((size_t)(restart + 2) * nr * z);
  char* nrm = take((size_t)nr * z);
  char* rho = take((size_t)nr * z);
  char* rhon = take((size_t)nr * z);
  char* pq = take((size_t)nr * z);
  char* alpha = take((size_t)nr * sizeof(double));
  char* beta = take((size_t)nr * sizeof(double));
  char* D = ir ? take((size_t)nr * N * z) : nullptr;
  char* Rr = ir ? take((size_t)nr * N * z) : nullptr;
  char* x32 = ir ? take((size_t)nr * CK * sizeof(float2)) : nullptr;
  char* y32 = ir ? take((size_t)nr * CK * sizeof(float2)) : nullptr;
  const size_t mvb = svh_workspace_bytes(p, SVH_FP64, nr);
  char* mv = take(mvb);
  const size_t mvb32 = ir ? svh_workspace_bytes(p, SVH_FP32, nr) : 0;
  char* mv32 = ir ? take(mvb32) : nullptr;
  if (w) {
    w->V = (double2*)V; w->Zk = (double2*)Zk; w->W = (double2*)W; w->Rhs = (double2*)Rhs;
    w->E = (double2*)E; w->R = (double2*)R; w->Zp = (double2*)Zp; w->P = (double2*)P; w->Q = (double2*)Q;
    w->Bs = (double2*)Bs; w->U = (double2*)U; w->part = (double2*)part; w->h = (double2*)h;
    w->h2 = (double2*)h2; w->nrm = (double2*)nrm; w->rho = (double2*)rho; w->rhon = (double2*)rhon;
    w->pq = (double2*)pq; w->alpha = (double*)alpha; w->beta = (double*)beta; w->mv = mv; w->mv_bytes = mvb;
    w->D = (double2*)D; w->Rr = (double2*)Rr; w->x32 = (float2*)x32; w->y32 = (float2*)y32;
    w->mv32 = mv32; w->mv32_bytes = mvb32;
  }
  return off;
}

struct Ctx {
  svh_problem* p;
  hipStream_t s;
  SolveWs w;
  int nr, CK, M, fidx, transpose;
  long long N;
  bool op32 = false;      // apply Z in FP32 (refinement inner solves)
  double t0 = 0;          // start of the solve (progress lines)
  hipGraphExec_t pcg_graph = nullptr;  // 16 PCG iterations, replayed
  hipGraph_t pcg_g = nullptr;
};

// out = sum over chunks of conj(X_(i,r)) Y_r into dst[(i * nr + r)]
void mdot(Ctx& c, long long n, int ni, const double2* X, long long xs_i, long long xs_r, const double2* Y,
          long long ys_r, double2* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_mdot, dim3(kDotBlocks, ni * c.nr), dim3(256), 0, s, n, c.nr, X, xs_i, xs_r, Y, ys_r,
                     c.w.part, 1);
  hipLaunchKernelGGL(k_psum, dim3(ni * c.nr), dim3(256), 0, s, kDotBlocks, c.w.part, dst);
}
void mdot(Ctx& c, long long n, int ni, const double2* X, long long xs_i, long long xs_r, const double2* Y,
          long long ys_r, double2* dst) {
  mdot(c, n, ni, X, xs_i, xs_r, Y, ys_r, dst, c.s);
}

__global__ void k_to32(int nrhs, long long N, int CK, const double2* __restrict__ x, float2* __restrict__ x32) {
  GRID_STRIDE(i, (long long)CK * nrhs) {
    const double2 v = x[(i / CK) * N + i % CK];
    x32[i] = make_float2((float)v.x, (float)v.y);
  }
}
__global__ void k_from32(int nrhs, long long N, int CK, const float2* __restrict__ y32, double2* __restrict__ y) {
  GRID_STRIDE(i, (long long)CK * nrhs) {
    const float2 v = y32[i];
    y[(i / CK) * N + i % CK] = make_double2(v.x, v.y);
  }
}

// y = K x (batched columns of length N); the Z block in FP32 when c.op32
svh_status apply_K(Ctx& c, const double2* x, double2* y) {
  svh_problem* p = c.p;
  std::vector<int32_t> fi(c.nr, c.fidx);
  svh_status st;
  if (c.op32) {
    const long long n = (long long)c.CK * c.nr;
    hipLaunchKernelGGL(k_to32, dim3(nblocks(n)), dim3(256), 0, c.s, c.nr, c.N, c.CK, x, c.w.x32);
    st = matvec_impl(p, SVH_FP32, c.nr, fi.data(), c.w.x32, c.CK, c.w.y32, c.CK, c.w.mv32, c.w.mv32_bytes, c.s);
    if (st != SVH_OK) return st;
    hipLaunchKernelGGL(k_from32, dim3(nblocks(n)), dim3(256), 0, c.s, c.nr, c.N, c.CK, c.w.y32, y);
  } else {
    st = matvec_impl(p, SVH_FP64, c.nr, fi.data(), x, c.N, y, c.N, c.w.mv, c.w.mv_bytes, c.s);
    if (st != SVH_OK) return st;
  }
  hipLaunchKernelGGL(k_saddle_fix, dim3(nblocks((c.CK + c.M) * (long long)c.nr)), dim3(256), 0, c.s, c.nr, c.N,
                     c.CK, c.M, p->d_cptr, p->d_crow, p->d_cval, p->d_rptr, p->d_rcol, p->d_rval, p->d_free, x, y,
                     c.transpose);
  SCHK(hipGetLastError());
  return SVH_OK;
}

constexpr int kPcgBlock = 16;  // PCG iterations per convergence check (one graph replay)

// One block of kPcgBlock conjugate-gradient iterations on S b = e, enqueued on s.
void vcycle(Ctx& c, const double2* b0, double2* x0, hipStream_t s);

void pcg_block(Ctx& c, hipStream_t s) {
  svh_problem* p = c.p;
  const long long nM = (long long)c.M * c.nr;
  for (int k = 0; k < kPcgBlock; ++k) {
    hipLaunchKernelGGL(k_s_half, dim3(resid_blocks(c.CK, c.nr)), dim3(256), 0, s, c.nr, c.CK, c.M,
                       p->d_cptr, p->d_crow, p->d_cval, p->d_ydiag, c.w.P, c.w.U);
    hipLaunchKernelGGL(k_s_full, dim3(resid_blocks(c.M, c.nr)), dim3(256), 0, s, c.nr, c.CK, c.M, p->d_rptr, p->d_rcol,
                       p->d_rval, p->d_free, c.w.U, c.w.Q);
    mdot(c, c.M, 1, c.w.P, 0, c.M, c.w.Q, c.M, c.w.pq, s);
    hipLaunchKernelGGL(k_pcg_alpha, dim3(1), dim3(256), 0, s, c.nr, c.w.rho, c.w.pq, c.w.alpha);
    hipLaunchKernelGGL(k_pcg_update, dim3(nblocks(nM)), dim3(256), 0, s, nM, c.M, p->d_sdiag, p->d_free,
                       c.w.alpha, c.w.P, c.w.Q, c.w.Bs, c.w.R, c.w.Zp);
    if (!p->amg.empty()) vcycle(c, c.w.R, c.w.Zp, s);
    mdot(c, c.M, 1, c.w.R, 0, c.M, c.w.Zp, c.M, c.w.rhon, s);
    hipLaunchKernelGGL(k_pcg_beta, dim3(1), dim3(256), 0, s, c.nr, c.w.rho, c.w.rhon, c.w.beta);
    hipLaunchKernelGGL(k_pcg_dir, dim3(nblocks(nM)), dim3(256), 0, s, nM, c.M, c.w.beta, c.w.Zp, c.w.P);
  }
}

// Capture pcg_block once per solve call (all pointers are fixed workspace
// buffers) on the problem's private stream; replays run on the caller's stream.
svh_status pcg_graph(Ctx& c) {
  svh_problem* p = c.p;
  if (c.pcg_graph || !p->use_graphs) return SVH_OK;
  if (!p->cap_stream) SCHK(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
  SCHK(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
  pcg_block(c, p->cap_stream);
  SCHK(hipStreamEndCapture(p->cap_stream, &c.pcg_g));
  SCHK(hipGraphInstantiate(&c.pcg_graph, c.pcg_g, nullptr, nullptr, 0));
  return SVH_OK;
}

// out = P in (eqs. 13-15), inner PCG to rel. tolerance itol; returns iterations
svh_status apply_P(Ctx& c, const double2* in, double2* out, double itol, int imax, int& iters) {
  svh_problem* p = c.p;
  const long long nM = (long long)c.M * c.nr;
  hipLaunchKernelGGL(k_pre_rhs, dim3(nblocks(nM)), dim3(256), 0, c.s, c.nr, c.N, c.CK, c.M, p->d_rptr, p->d_rcol,
                     p->d_rval, p->d_free, p->d_ydiag, in, c.w.E, c.transpose);
  hipLaunchKernelGGL(k_pcg_init, dim3(nblocks(nM)), dim3(256), 0, c.s, nM, c.M, p->d_sdiag, p->d_free, c.w.E,
                     c.w.R, c.w.Zp, c.w.P, c.w.Bs);
  if (!p->amg.empty()) {
    vcycle(c, c.w.R, c.w.Zp, c.s);
    hipLaunchKernelGGL(k_copy, dim3(nblocks(nM)), dim3(256), 0, c.s, nM, c.w.Zp, c.w.P);
  }
  mdot(c, c.M, 1, c.w.R, 0, c.M, c.w.Zp, c.M, c.w.rho);
  std::vector<double2> rho0(c.nr), rhoc(c.nr);
  SCHK(hipMemcpyAsync(rho0.data(), c.w.rho, sizeof(double2) * c.nr, hipMemcpyDeviceToHost, c.s));
  SCHK(hipStreamSynchronize(c.s));
  iters = 0;
  bool any = false;
  for (int r = 0; r < c.nr; ++r) any = any || rho0[r].x > 0;
  svh_status st = pcg_graph(c);
  if (st != SVH_OK) return st;
  while (any && iters < imax) {
    if (c.pcg_graph) SCHK(hipGraphLaunch(c.pcg_graph, c.s));
    else pcg_block(c, c.s);
    iters += kPcgBlock;
    SCHK(hipMemcpyAsync(rhoc.data(), c.w.rho, sizeof(double2) * c.nr, hipMemcpyDeviceToHost, c.s));
    SCHK(hipStreamSynchronize(c.s));
    any = false;
    for (int r = 0; r < c.nr; ++r)
      if (rho0[r].x > 0 && std::sqrt(std::max(rhoc[r].x, 0.0) / rho0[r].x) > itol) any = true;
  }
  hipLaunchKernelGGL(k_pre_out, dim3(nblocks((c.CK + c.M) * (long long)c.nr)), dim3(256), 0, c.s, c.nr, c.N, c.CK,
                     c.M, p->d_cptr, p->d_crow, p->d_cval, p->d_ydiag, in, c.w.Bs, out, c.transpose);
  SCHK(hipGetLastError());
  return SVH_OK;
}

// |diag Z| per basis function and the diagonal of S for frequency slot f
void free_amg(svh_problem* p) {
  for (auto& L : p->amg) {
    fr(L.rptr);
    fr(L.col);
    fr(L.val);
    fr(L.dinv);
    fr(L.agg);
    fr(L.mptr);
    fr(L.mem);
    fr(L.b);
    fr(L.x);
    fr(L.r);
  }
  p->amg.clear();
  fr(p->d_amg_cinv);
}

// Multigrid hierarchy of S for the current Y and Dirichlet set, with work
// vectors for nports right-hand sides.
svh_status build_amg(svh_problem* p, const std::vector<double>& yd) {
  free_amg(p);
  std::vector<AmgLevel> levels;
  std::vector<std::vector<int>> aggs;
  std::vector<double> cinv;
  const int kind = amg_setup(schur_matrix(p->topo, p->dirichlet, yd), levels, aggs, cinv);
  if (kind < 0) return sfail(p, SVH_EINVAL, "solve: multigrid setup of the Schur complement failed");
  p->amg_coarse = kind;
  const int nr = p->nports;
  p->amg.resize(levels.size());
  for (size_t l = 0; l < levels.size(); ++l) {
    const AmgLevel& L = levels[l];
    auto& D = p->amg[l];
    D.n = L.n;
    std::vector<double> dinv(L.n, 1.0);
    for (int i = 0; i < L.n; ++i) {
      bool coupled = false;
      double dg = 0;
      for (int q = L.rptr[i]; q < L.rptr[i + 1]; ++q) {
        if (L.col[q] == i) dg = L.val[q];
        else if (L.val[q] != 0) coupled = true;
      }
      dinv[i] = dg > 0 ? (coupled ? kAmgOmega : 1.0) / dg : 1.0;
    }
    SCHK(up(&D.rptr, L.rptr.data(), L.rptr.size()));
    SCHK(up(&D.col, L.col.data(), L.col.size()));
    SCHK(up(&D.val, L.val.data(), L.val.size()));
    SCHK(up(&D.dinv, dinv.data(), dinv.size()));
    SCHK(hipMalloc(&D.r, sizeof(double2) * (size_t)nr * L.n));
    if (l > 0) {
      SCHK(hipMalloc(&D.b, sizeof(double2) * (size_t)nr * L.n));
      SCHK(hipMalloc(&D.x, sizeof(double2) * (size_t)nr * L.n));
    }
    if (l + 1 < levels.size()) {
      const std::vector<int>& agg = aggs[l];
      const int nc = levels[l + 1].n;
      std::vector<int> mptr(nc + 1, 0);
      for (int i = 0; i < L.n; ++i)
        if (agg[i] >= 0) mptr[agg[i] + 1]++;
      std::partial_sum(mptr.begin(), mptr.end(), mptr.begin());
      std::vector<int> mem(std::max(mptr[nc], 1), 0);
      std::vector<int> fill(mptr.begin(), mptr.end() - 1);
      for (int i = 0; i < L.n; ++i)
        if (agg[i] >= 0) mem[fill[agg[i]]++] = i;
      SCHK(up(&D.agg, agg.data(), agg.size()));
      SCHK(up(&D.mptr, mptr.data(), mptr.size()));
      SCHK(up(&D.mem, mem.data(), mem.size()));
    }
  }
  if (!cinv.empty()) SCHK(up(&p->d_amg_cinv, cinv.data(), cinv.size()));
  p->amg_nr = nr;
  return SVH_OK;
}

// z = B r: one symmetric V-cycle (one damped-Jacobi sweep before and after
// the scaled coarse correction; on the coarsest level its dense inverse, its
// diagonal when it has no couplings, or damped Jacobi sweeps) per right-hand
// side.
void vcycle(Ctx& c, const double2* b0, double2* x0, hipStream_t s) {
  svh_problem* p = c.p;
  const int nl = (int)p->amg.size(), nr = c.nr;
  for (int l = 0; l < nl; ++l) {
    auto& L = p->amg[l];
    const double2* b = l ? L.b : b0;
    double2* x = l ? L.x : x0;
    const long long n = (long long)L.n * nr;
    if (l == nl - 1) {
      if (p->amg_coarse == kAmgCoarseDense) {
        hipLaunchKernelGGL(k_amg_coarse, dim3(nblocks(n)), dim3(256), 0, s, nr, L.n, p->d_amg_cinv, b, x);
      } else {  // diagonal matrix (exact), or damped Jacobi sweeps
        hipLaunchKernelGGL(k_amg_smooth0, dim3(nblocks(n)), dim3(256), 0, s, nr, L.n, L.dinv, b, x);
        for (int k = 1; k < (p->amg_coarse == kAmgCoarseJacobi ? kAmgCoarseSweeps : 1); ++k) {
          amg_resid(L, nr, b, x, L.r, s);
          hipLaunchKernelGGL(k_amg_jacobi, dim3(nblocks(n)), dim3(256), 0, s, nr, L.n, L.dinv, L.r, x);
        }
      }
      break;
    }
    hipLaunchKernelGGL(k_amg_smooth0, dim3(nblocks(n)), dim3(256), 0, s, nr, L.n, L.dinv, b, x);
    amg_resid(L, nr, b, x, L.r, s);
    auto& Cl = p->amg[l + 1];
    hipLaunchKernelGGL(k_amg_restrict, dim3(nblocks((long long)Cl.n * nr)), dim3(256), 0, s, nr, L.n, Cl.n, L.mptr,
                       L.mem, L.r, Cl.b);
  }
  for (int l = nl - 2; l >= 0; --l) {
    auto& L = p->amg[l];
    auto& Cl = p->amg[l + 1];
    const double2* b = l ? L.b : b0;
    double2* x = l ? L.x : x0;
    const long long n = (long long)L.n * nr;
    hipLaunchKernelGGL(k_amg_prolong, dim3(nblocks(n)), dim3(256), 0, s, nr, L.n, Cl.n, L.agg, Cl.x, x);
    amg_resid(L, nr, b, x, L.r, s);
    hipLaunchKernelGGL(k_amg_jacobi, dim3(nblocks(n)), dim3(256), 0, s, nr, L.n, L.dinv, L.r, x);
  }
}

svh_status prepare_diag(svh_problem* p, int f) {
  if (p->diag_freq == f && p->d_ydiag) return SVH_OK;
  const int K = p->nvox, CK = p->C * K, M = p->topo.M;
  const std::complex<double> s = p->sconv[f];  // j w mu0 dx
  // self block of each basis function at offset 0 (eq. 8): M0 for the
  // constant ones, M2x + M2y and M2x + M2y + 4 M2z for the linear ones, and
  // its mass weight 1, 1/6, 1/2
  double self[5] = {p->T[0], p->T[0], p->T[0], 0, 0};
  const double mass[5] = {1.0, 1.0, 1.0, 1.0 / 6.0, 0.5};
  if (p->C == 5) {
    const size_t Kt = (size_t)p->K[0] * p->K[1] * p->K[2];
    const double m2x = p->Tf[4 * Kt], m2y = p->Tf[5 * Kt], m2z = p->Tf[6 * Kt];
    self[3] = m2x + m2y;
    self[4] = m2x + m2y + 4 * m2z;
  }
  std::vector<double> yd(CK), sd(M, 1.0);
  for (int a = 0; a < p->C; ++a)
    for (int k = 0; k < K; ++k)
      yd[(size_t)a * K + k] = std::abs(mass[a] * p->cdiag_host[(size_t)f * K + k] + s * self[a]);
  for (int m = 0; m < M; ++m) {
    if (p->dirichlet[m]) continue;
    double acc = 0;
    for (int q = p->topo.rptr[m]; q < p->topo.rptr[m + 1]; ++q)
      acc += p->topo.rval[q] * p->topo.rval[q] / yd[p->topo.rcol[q]];
    sd[m] = acc > 0 ? acc : 1.0;
  }
  SCHK(up(&p->d_ydiag, yd.data(), yd.size()));
  SCHK(up(&p->d_sdiag, sd.data(), sd.size()));
  p->diag_freq = f;
  if (p->schur_precond == SVH_SCHUR_AMG) return build_amg(p, yd);
  free_amg(p);
  return SVH_OK;
}

// complex Givens rotation zeroing b below a (b real >= 0)
void givens(cd a, double b, double& cs, cd& sn, cd& r) {
  const double aa = std::abs(a);
  if (aa == 0) {
    cs = 0;
    sn = 1;
    r = b;
    return;
  }
  const double rho = std::sqrt(aa * aa + b * b);
  cs = aa / rho;
  sn = (a / aa) * b / rho;
  r = (a / aa) * rho;
}

struct FgmresStats {
  int total = 0, inner = 0, restarts = 0;
};

svh_status finish(Ctx& c, svh_status st) {
  if (c.pcg_graph) (void)hipGraphExecDestroy(c.pcg_graph);
  if (c.pcg_g) (void)hipGraphDestroy(c.pcg_g);
  c.pcg_graph = nullptr;
  c.pcg_g = nullptr;
  return st;
}

// per-column 2-norms of a batch of N-vectors
svh_status norms(Ctx& c, const double2* v, std::vector<double>& out) {
  svh_problem* p = c.p;
  mdot(c, c.N, 1, v, 0, c.N, v, c.N, c.w.nrm);
  std::vector<double2> h(c.nr);
  SCHK(hipMemcpyAsync(h.data(), c.w.nrm, sizeof(double2) * c.nr, hipMemcpyDeviceToHost, c.s));
  SCHK(hipStreamSynchronize(c.s));
  out.resize(c.nr);
  for (int r = 0; r < c.nr; ++r) out[r] = std::sqrt(std::max(h[r].x, 0.0));
  return SVH_OK;
}

// Right-preconditioned flexible GMRES(restart) on K X = B for every column,
// starting from the X given; stops when every column's residual estimate is
// below rre * bnorm[r] or after maxit steps.
svh_status fgmres(Ctx& c, const double2* B, double2* X, const std::vector<double>& bnorm, double rre, int restart,
                  int maxit, double itol, FgmresStats& fs, int max_cycles = 1 << 30) {
  svh_problem* p = c.p;
  const int nr = c.nr;
  const long long NN = c.N * nr;
  const long long vs = NN;  // stride between Krylov vectors
  const int imax = 20000;
  svh_status st;
  int steps = 0, cycles = 0;
  bool first = true;
  while (steps < maxit && cycles < max_cycles) {
    if (first) {
      hipLaunchKernelGGL(k_copy, dim3(nblocks(NN)), dim3(256), 0, c.s, NN, B, c.w.W);
      hipLaunchKernelGGL(k_zero, dim3(nblocks(NN)), dim3(256), 0, c.s, NN, X);
      first = false;
    } else {
      if ((st = apply_K(c, X, c.w.W)) != SVH_OK) return st;
      hipLaunchKernelGGL(k_resid, dim3(nblocks(NN)), dim3(256), 0, c.s, NN, B, c.w.W);
    }
    std::vector<double> beta;
    if ((st = norms(c, c.w.W, beta)) != SVH_OK) return st;
    bool done = true;
    for (int r = 0; r < nr; ++r)
      if (bnorm[r] > 0 && beta[r] > rre * bnorm[r]) done = false;
    if (done) return SVH_OK;
    hipLaunchKernelGGL(k_normalize, dim3(nblocks(NN)), dim3(256), 0, c.s, c.N, nr, c.w.nrm, c.w.W, c.w.V);
    std::vector<std::vector<cd>> H(nr, std::vector<cd>((size_t)(restart + 1) * restart, 0.0));
    std::vector<std::vector<double>> cs(nr, std::vector<double>(restart, 0.0));
    std::vector<std::vector<cd>> sn(nr, std::vector<cd>(restart, 0.0));
    std::vector<std::vector<cd>> g(nr, std::vector<cd>(restart + 1, 0.0));
    for (int r = 0; r < nr; ++r) g[r][0] = beta[r];
    int jdone = 0;
    std::vector<double2> hcol((size_t)(restart + 2) * nr);
    for (int j = 0; j < restart && steps < maxit; ++j) {
      int it = 0;
      if ((st = apply_P(c, c.w.V + j * vs, c.w.Zk + j * vs, itol, imax, it)) != SVH_OK) return st;
      fs.inner += it;
      if ((st = apply_K(c, c.w.Zk + j * vs, c.w.W)) != SVH_OK) return st;
      // CGS2
      mdot(c, c.N, j + 1, c.w.V, vs, c.N, c.w.W, c.N, c.w.h);
      hipLaunchKernelGGL(k_cgs_update, dim3(nblocks(NN)), dim3(256), 0, c.s, c.N, nr, j + 1, c.w.V, vs, c.w.h,
                         c.w.W);
      mdot(c, c.N, j + 1, c.w.V, vs, c.N, c.w.W, c.N, c.w.h2);
      hipLaunchKernelGGL(k_cgs_update, dim3(nblocks(NN)), dim3(256), 0, c.s, c.N, nr, j + 1, c.w.V, vs, c.w.h2,
                         c.w.W);
      hipLaunchKernelGGL(k_add_small, dim3(((j + 1) * nr + 255) / 256), dim3(256), 0, c.s, (j + 1) * nr, c.w.h,
                         c.w.h2);
      mdot(c, c.N, 1, c.w.W, 0, c.N, c.w.W, c.N, c.w.nrm);
      hipLaunchKernelGGL(k_normalize, dim3(nblocks(NN)), dim3(256), 0, c.s, c.N, nr, c.w.nrm, c.w.W,
                         c.w.V + (j + 1) * vs);
      SCHK(hipMemcpyAsync(hcol.data(), c.w.h, sizeof(double2) * (j + 1) * nr, hipMemcpyDeviceToHost, c.s));
      SCHK(hipMemcpyAsync(hcol.data() + (size_t)(j + 1) * nr, c.w.nrm, sizeof(double2) * nr,
                          hipMemcpyDeviceToHost, c.s));
      SCHK(hipStreamSynchronize(c.s));
      ++steps;
      ++fs.total;
      jdone = j + 1;
      bool all = true;
      for (int r = 0; r < nr; ++r) {
        std::vector<cd>& Hr = H[r];
        for (int i = 0; i <= j; ++i)
          Hr[(size_t)i * restart + j] = cd(hcol[(size_t)i * nr + r].x, hcol[(size_t)i * nr + r].y);
        const double hj1 = std::sqrt(std::max(hcol[(size_t)(j + 1) * nr + r].x, 0.0));
        for (int i = 0; i < j; ++i) {
          const cd a = Hr[(size_t)i * restart + j], b = Hr[(size_t)(i + 1) * restart + j];
          Hr[(size_t)i * restart + j] = cs[r][i] * a + sn[r][i] * b;
          Hr[(size_t)(i + 1) * restart + j] = -std::conj(sn[r][i]) * a + cs[r][i] * b;
        }
        cd rr;
        givens(Hr[(size_t)j * restart + j], hj1, cs[r][j], sn[r][j], rr);
        Hr[(size_t)j * restart + j] = rr;
        const cd gj = g[r][j];
        g[r][j] = cs[r][j] * gj;
        g[r][j + 1] = -std::conj(sn[r][j]) * gj;
        if (bnorm[r] > 0 && std::abs(g[r][j + 1]) > rre * bnorm[r]) all = false;
      }
      if (all) break;
    }
    // y = H^-1 g, x += Zk y
    std::vector<double2> coef((size_t)jdone * nr);
    for (int r = 0; r < nr; ++r) {
      std::vector<cd> y(jdone);
      for (int i = jdone - 1; i >= 0; --i) {
        cd acc = g[r][i];
        for (int k = i + 1; k < jdone; ++k) acc -= H[r][(size_t)i * restart + k] * y[k];
        const cd d = H[r][(size_t)i * restart + i];
        y[i] = std::abs(d) > 0 ? acc / d : cd(0.0);
      }
      for (int i = 0; i < jdone; ++i) coef[(size_t)i * nr + r] = make_double2(y[i].real(), y[i].imag());
    }
    SCHK(hipMemcpyAsync(c.w.h2, coef.data(), sizeof(double2) * coef.size(), hipMemcpyHostToDevice, c.s));
    hipLaunchKernelGGL(k_combine, dim3(nblocks(NN)), dim3(256), 0, c.s, c.N, nr, jdone, c.w.Zk, vs, c.w.h2, X);
    ++fs.restarts;
    ++cycles;
    SCHK(hipStreamSynchronize(c.s));
    if (verbose(p)) {
      double worst = 0;
      for (int r = 0; r < nr; ++r)
        if (bnorm[r] > 0) worst = std::max(worst, std::abs(g[r][jdone]) / bnorm[r]);
      std::fprintf(stderr, "[svh] fgmres cycle %d (%s): %d steps, estimate %.3e, inner CG steps %d, %.2f s\n",
                   cycles, c.op32 ? "fp32 operator" : "fp64", fs.total, worst, fs.inner, now_s() - c.t0);
      std::fflush(stderr);
    }
  }
  return SVH_ENOTCONV;
}

// Z = A^-1 for a small dense complex matrix (row-major n x n), Gauss-Jordan
// elimination with partial pivoting; false if A is singular.
bool invert_small(int n, std::vector<cd> A, std::vector<cd>& Z) {
  Z.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
  double amax = 0;
  for (const cd& v : A) amax = std::max(amax, std::abs(v));
  if (!(amax > 0)) return false;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::abs(A[(size_t)r * n + c]) > std::abs(A[(size_t)piv * n + c])) piv = r;
    if (!(std::abs(A[(size_t)piv * n + c]) > 1e-300 * amax)) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(A[(size_t)piv * n + k], A[(size_t)c * n + k]);
        std::swap(Z[(size_t)piv * n + k], Z[(size_t)c * n + k]);
      }
    const cd inv = 1.0 / A[(size_t)c * n + c];
    for (int k = 0; k < n; ++k) {
      A[(size_t)c * n + k] *= inv;
      Z[(size_t)c * n + k] *= inv;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const cd f = A[(size_t)r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        A[(size_t)r * n + k] -= f * A[(size_t)c * n + k];
        Z[(size_t)r * n + k] -= f * Z[(size_t)c * n + k];
      }
    }
  }
  return true;
}

// w of frequency slot f (the coupling scalar is j w mu0 dx)
double angular_frequency(const svh_problem* p, int f) { return p->sconv[f].imag() / (kMu0 * p->dx); }

}  // namespace

void free_solver(svh_problem* p) {
  fr(p->d_cptr);
  fr(p->d_crow);
  fr(p->d_cval);
  fr(p->d_rptr);
  fr(p->d_rcol);
  fr(p->d_rval);
  fr(p->d_free);
  fr(p->d_bport);
  fr(p->d_ydiag);
  fr(p->d_sdiag);
  free_amg(p);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  p->cap_stream = nullptr;
}

}  // namespace svh

using namespace svh;

extern "C" {

svh_status svh_set_ports(svh_problem* p, int nports, const int32_t* plus_ptr, const int32_t* plus_faces,
                         const int32_t* minus_ptr, const int32_t* minus_faces) {
  if (!p) return SVH_EINVAL;
  if (nports < 1 || nports > SVH_MAX_PORTS || !plus_ptr || !plus_faces || !minus_ptr || !minus_faces)
    return sfail(p, SVH_EINVAL, "set_ports: bad arguments");
  if (!p->topo_built) {
    if (build_topology(p->K, p->vidx.data(), p->nvox, p->basis, p->topo) != 0)
      return sfail(p, SVH_EINVAL, "set_ports: unsupported basis");
    p->topo_built = true;
    SCHK(up(&p->d_cptr, p->topo.cptr.data(), p->topo.cptr.size()));
    SCHK(up(&p->d_crow, p->topo.crow.data(), p->topo.crow.size()));
    SCHK(up(&p->d_cval, p->topo.cval.data(), p->topo.cval.size()));
    SCHK(up(&p->d_rptr, p->topo.rptr.data(), p->topo.rptr.size()));
    SCHK(up(&p->d_rcol, p->topo.rcol.data(), p->topo.rcol.size()));
    SCHK(up(&p->d_rval, p->topo.rval.data(), p->topo.rval.size()));
  }
  const int M = p->topo.M, K = p->nvox, CK = p->C * K;
  std::vector<char> dir(M, 0);
  std::vector<std::vector<int>> plus(nports);
  auto node_of = [&](int k, int face, int& m) -> bool {
    if (k < 0 || k >= K || face < 0 || face > 5) return false;
    m = p->topo.face_node[6 * (size_t)k + face];
    return m >= 0;
  };
  for (int q = 0; q < nports; ++q) {
    if (plus_ptr[q + 1] <= plus_ptr[q] || minus_ptr[q + 1] <= minus_ptr[q])
      return sfail(p, SVH_EINVAL, "set_ports: every port needs + and - faces");
    for (int i = plus_ptr[q]; i < plus_ptr[q + 1]; ++i) {
      int m;
      if (!node_of(plus_faces[2 * i], plus_faces[2 * i + 1], m)) return sfail(p, SVH_EINVAL, "set_ports: bad face");
      plus[q].push_back(m);
      dir[m] = 1;
    }
    for (int i = minus_ptr[q]; i < minus_ptr[q + 1]; ++i) {
      int m;
      if (!node_of(minus_faces[2 * i], minus_faces[2 * i + 1], m)) return sfail(p, SVH_EINVAL, "set_ports: bad face");
      dir[m] = 1;
    }
  }
  ground_floating(p->topo, dir);
  p->dirichlet = dir;
  p->port_plus = plus;
  p->nports = nports;
  // b_q = A_{q+}^T 1 (one value per basis function)
  std::vector<char> inplus(M, 0);
  p->bport_host.assign((size_t)nports * CK, 0.0);
  for (int q = 0; q < nports; ++q) {
    for (int m : plus[q]) inplus[m] = 1;
    for (int col = 0; col < CK; ++col)
      for (int i = p->topo.cptr[col]; i < p->topo.cptr[col + 1]; ++i)
        if (inplus[p->topo.crow[i]]) p->bport_host[(size_t)q * CK + col] += p->topo.cval[i];
    for (int m : plus[q]) inplus[m] = 0;
  }
  std::vector<uint8_t> fm(M);
  for (int m = 0; m < M; ++m) fm[m] = dir[m] ? 0 : 1;
  SCHK(up(&p->d_free, fm.data(), fm.size()));
  SCHK(up(&p->d_bport, p->bport_host.data(), p->bport_host.size()));
  p->diag_freq = -2;
  return SVH_OK;
}

svh_status svh_solve_sizes(const svh_problem* p, int* N, int* M) {
  if (!p || !p->topo_built) return SVH_ESTATE;
  if (M) *M = p->topo.M;
  if (N) *N = p->C * p->nvox + p->topo.M;
  return SVH_OK;
}

size_t svh_solve_workspace_bytes(const svh_problem* p, svh_prec prec, int restart) {
  if (!p || !p->topo_built || restart < 1 || (prec != SVH_FP64 && prec != SVH_FP32_IR)) return 0;
  return carve(p, restart, prec, nullptr, nullptr) + 1024;
}

svh_status svh_solve(svh_problem* p, svh_prec prec, int freq_idx, double rre, int restart, int maxit,
                     int transpose, void* x_dev, double* Y_host, svh_solve_info* info, void* ws, size_t ws_bytes,
                     void* stream) {
  if (!p) return SVH_EINVAL;
  if (!p->topo_built || p->nports < 1) return sfail(p, SVH_ESTATE, "solve: set the ports first");
  if (p->T.empty() || p->nfreq < 1) return sfail(p, SVH_ESTATE, "solve: set material and tensors first");
  if (prec != SVH_FP64 && prec != SVH_FP32_IR) return sfail(p, SVH_EINVAL, "solve: precision not supported");
  if (freq_idx < 0 || freq_idx >= p->nfreq || !(rre > 0) || restart < 1 || maxit < 1 || !x_dev || !ws)
    return sfail(p, SVH_EINVAL, "solve: bad arguments");
  if (ws_bytes < svh_solve_workspace_bytes(p, prec, restart))
    return sfail(p, SVH_EINVAL, "solve: workspace too small");
  Ctx c;
  c.p = p;
  c.s = static_cast<hipStream_t>(stream);
  c.nr = p->nports;
  c.CK = p->C * p->nvox;
  c.M = p->topo.M;
  c.N = (long long)c.CK + c.M;
  c.fidx = freq_idx;
  c.transpose = transpose ? 1 : 0;
  c.t0 = now_s();
  carve(p, restart, prec, static_cast<char*>((void*)(((uintptr_t)ws + 255) & ~(uintptr_t)255)), &c.w);
  svh_status st = prepare_diag(p, freq_idx);
  if (st != SVH_OK) return st;
  if (verbose(p)) {
    std::fprintf(stderr, "[svh] solve: N = %lld per port, %d ports, %s, multigrid levels %zu, set-up %.2f s\n",
                 c.N, c.nr, prec == SVH_FP64 ? "fp64" : "fp32 operator + fp64 refinement", p->amg.size(),
                 now_s() - c.t0);
    std::fflush(stderr);
  }
  const int nr = c.nr;
  const long long NN = c.N * nr;
  double2* X = static_cast<double2*>(x_dev);
  hipLaunchKernelGGL(k_port_rhs, dim3(nblocks(NN)), dim3(256), 0, c.s, nr, c.N, c.CK, p->d_bport, c.w.Rhs);
  hipLaunchKernelGGL(k_zero, dim3(nblocks(NN)), dim3(256), 0, c.s, NN, X);
  std::vector<double> bnorm;
  if ((st = norms(c, c.w.Rhs, bnorm)) != SVH_OK) return finish(c, st);
  FgmresStats fs;
  int ir_steps = 0;
  std::vector<double> relres(nr, 1.0);
  if (prec == SVH_FP64) {
    c.op32 = false;
    st = fgmres(c, c.w.Rhs, X, bnorm, rre, restart, maxit, p->schur_tol > 0 ? p->schur_tol : std::min(1e-8, rre), fs);
    if (st != SVH_OK && st != SVH_ENOTCONV) return finish(c, st);
  } else {
    // iterative refinement: FP64 residual, FP32 operator in the inner solve
    hipLaunchKernelGGL(k_copy, dim3(nblocks(NN)), dim3(256), 0, c.s, NN, c.w.Rhs, c.w.Rr);
    std::vector<double> rn = bnorm;
    const double inner = std::max(1e-6, rre);
    for (ir_steps = 0; ir_steps < 30 && fs.total < maxit; ++ir_steps) {
      bool done = true;
      for (int r = 0; r < nr; ++r)
        if (bnorm[r] > 0 && rn[r] / bnorm[r] > rre) done = false;
      if (done) break;
      hipLaunchKernelGGL(k_zero, dim3(nblocks(NN)), dim3(256), 0, c.s, NN, c.w.D);
      c.op32 = true;
      // one inner cycle per refinement step, judged by its own recurrence
      // estimate; only the FP64 residual below decides convergence (a true
      // residual formed with the FP32 operator would stall at its rounding floor)
      // inner target: the remaining factor to the goal, at least 1e-6 (FP32)
      double need = 1.0;
      for (int r = 0; r < nr; ++r)
        if (rn[r] > 0) need = std::min(need, rre * bnorm[r] / rn[r]);
      const double tin = std::max(inner, need);
      st = fgmres(c, c.w.Rr, c.w.D, rn, tin, restart, maxit - fs.total,
                  p->schur_tol > 0 ? p->schur_tol : std::min(1e-8, tin * 1e-2), fs, 1);
      if (st != SVH_OK && st != SVH_ENOTCONV) return finish(c, st);
      hipLaunchKernelGGL(k_add, dim3(nblocks(NN)), dim3(256), 0, c.s, NN, c.w.D, X);
      c.op32 = false;
      if ((st = apply_K(c, X, c.w.Rr)) != SVH_OK) return finish(c, st);
      hipLaunchKernelGGL(k_resid, dim3(nblocks(NN)), dim3(256), 0, c.s, NN, c.w.Rhs, c.w.Rr);
      if ((st = norms(c, c.w.Rr, rn)) != SVH_OK) return finish(c, st);
      if (verbose(p)) {
        double worst = 0;
        for (int r = 0; r < nr; ++r)
          if (bnorm[r] > 0) worst = std::max(worst, rn[r] / bnorm[r]);
        std::fprintf(stderr, "[svh] refinement step %d: fp64 residual %.3e, %.2f s\n", ir_steps + 1, worst,
                     now_s() - c.t0);
        std::fflush(stderr);
      }
    }
  }
  // true FP64 residual
  c.op32 = false;
  if ((st = apply_K(c, X, c.w.W)) != SVH_OK) return finish(c, st);
  hipLaunchKernelGGL(k_resid, dim3(nblocks(NN)), dim3(256), 0, c.s, NN, c.w.Rhs, c.w.W);
  std::vector<double> rfin;
  if ((st = norms(c, c.w.W, rfin)) != SVH_OK) return finish(c, st);
  // port admittance Y[q][p] = b_q^T I_p
  std::vector<double2> yq((size_t)nr * nr);
  hipLaunchKernelGGL(k_ydot, dim3(kDotBlocks, nr * nr), dim3(256), 0, c.s, c.CK, nr, c.N, p->d_bport, X, c.w.part);
  hipLaunchKernelGGL(k_psum, dim3(nr * nr), dim3(256), 0, c.s, kDotBlocks, c.w.part, c.w.V);
  SCHK(hipMemcpyAsync(yq.data(), c.w.V, sizeof(double2) * yq.size(), hipMemcpyDeviceToHost, c.s));
  SCHK(hipStreamSynchronize(c.s));
  double worst = 0;
  for (int r = 0; r < nr; ++r) {
    relres[r] = bnorm[r] > 0 ? rfin[r] / bnorm[r] : 0.0;
    worst = std::max(worst, relres[r]);
  }
  const bool converged = worst <= 2 * rre;  // true residual, with slack for rounding
  if (Y_host)
    for (size_t i = 0; i < yq.size(); ++i) {
      Y_host[2 * i] = yq[i].x;
      Y_host[2 * i + 1] = yq[i].y;
    }
  if (info) {
    info->iterations = fs.total;
    info->restarts = fs.restarts;
    info->inner_iterations = fs.inner;
    info->refinement_steps = ir_steps;
    info->relres = worst;
    for (int r = 0; r < nr && r < SVH_MAX_PORTS; ++r) info->relres_port[r] = relres[r];
    info->converged = converged ? 1 : 0;
  }
  return finish(c, converged ? SVH_OK : SVH_ENOTCONV);
}

svh_status svh_port_gradient(svh_problem* p, int freq_idx, const void* xfwd_dev, const void* xadj_dev,
                             void* dY_dev, void* stream) {
  if (!p) return SVH_EINVAL;
  if (!p->topo_built || p->nports < 1) return sfail(p, SVH_ESTATE, "port_gradient: set the ports first");
  if (freq_idx < 0 || freq_idx >= p->nfreq || !xfwd_dev || !xadj_dev || !dY_dev)
    return sfail(p, SVH_EINVAL, "port_gradient: bad arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int K = p->nvox, nr = p->nports;
  const long long N = (long long)p->C * K + p->topo.M;
  const double w = angular_frequency(p, freq_idx);
  const double inv_wmu = p->dx / (w * kMu0);
  hipLaunchKernelGGL(k_port_grad, dim3(nblocks((long long)K * nr * nr)), dim3(256), 0, s, nr, p->C, K, N,
                     p->d_cdiag64 + (size_t)freq_idx * K, inv_wmu, static_cast<const double2*>(xfwd_dev),
                     static_cast<const double2*>(xadj_dev), static_cast<double2*>(dY_dev));
  SCHK(hipGetLastError());
  return SVH_OK;
}

svh_status svh_port_inductance(svh_problem* p, int freq_idx, const double* Y_host, double* Z_host, double* L_host) {
  if (!p) return SVH_EINVAL;
  if (p->nports < 1 || !Y_host) return sfail(p, SVH_EINVAL, "port_inductance: bad arguments (set the ports first)");
  if (freq_idx < 0 || freq_idx >= p->nfreq) return sfail(p, SVH_EINVAL, "port_inductance: bad frequency slot");
  const int n = p->nports;
  std::vector<cd> Y((size_t)n * n), Z;
  for (size_t i = 0; i < Y.size(); ++i) Y[i] = cd(Y_host[2 * i], Y_host[2 * i + 1]);
  if (!invert_small(n, Y, Z)) return sfail(p, SVH_EINVAL, "port_inductance: singular admittance matrix");
  const double w = angular_frequency(p, freq_idx);
  for (size_t i = 0; i < Z.size(); ++i) {
    if (Z_host) {
      Z_host[2 * i] = Z[i].real();
      Z_host[2 * i + 1] = Z[i].imag();
    }
    if (L_host) L_host[i] = Z[i].imag() / w;
  }
  return SVH_OK;
}

svh_status svh_gradient_contract(svh_problem* p, int freq_idx, const double* Y_host, const double* G_host,
                                 const void* dY_dev, double* grad_dev, void* ws_dev, size_t ws_bytes, void* stream) {
  if (!p) return SVH_EINVAL;
  if (p->nports < 1 || !Y_host || !G_host || !dY_dev || !grad_dev || !ws_dev)
    return sfail(p, SVH_EINVAL, "gradient_contract: bad arguments");
  if (freq_idx < 0 || freq_idx >= p->nfreq) return sfail(p, SVH_EINVAL, "gradient_contract: bad frequency slot");
  const int n = p->nports;
  if (ws_bytes < sizeof(double2) * n * n) return sfail(p, SVH_EINVAL, "gradient_contract: workspace too small");
  std::vector<cd> Y((size_t)n * n), Z;
  for (size_t i = 0; i < Y.size(); ++i) Y[i] = cd(Y_host[2 * i], Y_host[2 * i + 1]);
  if (!invert_small(n, Y, Z)) return sfail(p, SVH_EINVAL, "gradient_contract: singular admittance matrix");
  // Loss = sum_qp G_qp L_qp with L = Im(Z) / w and dZ = -Z dY Z, so
  // dLoss/dp_k = -(1/w) Im( sum_ab W_ab dY_ab ), W = Z^T G Z^T
  std::vector<cd> T((size_t)n * n, 0.0);
  std::vector<double2> W((size_t)n * n);
  for (int a = 0; a < n; ++a)  // T = Z^T G
    for (int pp = 0; pp < n; ++pp) {
      cd acc = 0;
      for (int q = 0; q < n; ++q) acc += Z[(size_t)q * n + a] * G_host[(size_t)q * n + pp];
      T[(size_t)a * n + pp] = acc;
    }
  for (int a = 0; a < n; ++a)  // W = T Z^T
    for (int b = 0; b < n; ++b) {
      cd acc = 0;
      for (int pp = 0; pp < n; ++pp) acc += T[(size_t)a * n + pp] * Z[(size_t)b * n + pp];
      W[(size_t)a * n + b] = make_double2(acc.real(), acc.imag());
    }
  const double w = angular_frequency(p, freq_idx);
  hipStream_t s = static_cast<hipStream_t>(stream);
  double2* dW = static_cast<double2*>(ws_dev);
  SCHK(hipMemcpyAsync(dW, W.data(), sizeof(double2) * n * n, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_grad_contract, dim3(nblocks(p->nvox)), dim3(256), 0, s, n, p->nvox, dW,
                     static_cast<const double2*>(dY_dev), -1.0 / w, grad_dev);
  SCHK(hipGetLastError());
  SCHK(hipStreamSynchronize(s));  // W lives on this frame
  return SVH_OK;
}

svh_status svh_matvec_adjoint(svh_problem* p, svh_prec prec, int nrhs, const int32_t* freq_idx_host,
                              const void* x_dev, void* y_dev, void* ws_dev, size_t ws_bytes, void* stream) {
  // The Galerkin blocks satisfy B^{alpha beta}(-d) = B^{beta alpha}(d): the
  // constant-basis blocks depend on the offset through the even M0, and a
  // block with an odd M1 family changes sign both under d -> -d and under the
  // exchange of the two basis functions (eq. 8: (x, 2D) = +M1x, (2D, x) =
  // -M1x).  The diagonal is symmetric, so Z^T = Z (transpose, not conjugate)
  // and the transposed block table is the block table itself: the adjoint
  // product runs the same kernels.
  if (!p) return SVH_EINVAL;
  return svh_matvec(p, prec, nrhs, freq_idx_host, x_dev, y_dev, ws_dev, ws_bytes, stream);
}

svh_status svh_set_schur_precond(svh_problem* p, int kind) {
  if (!p) return SVH_EINVAL;
  if (kind != SVH_SCHUR_JACOBI && kind != SVH_SCHUR_AMG) return sfail(p, SVH_EINVAL, "set_schur_precond: unknown kind");
  if (kind != p->schur_precond) p->diag_freq = -2;  // rebuilt at the next solve
  p->schur_precond = kind;
  return SVH_OK;
}

svh_status svh_set_schur_tol(svh_problem* p, double tol) {
  if (!p) return SVH_EINVAL;
  if (!(tol >= 0) || !(tol < 1)) return sfail(p, SVH_EINVAL, "set_schur_tol: need 0 <= tol < 1");
  p->schur_tol = tol;
  return SVH_OK;
}

svh_status svh_set_graphs(svh_problem* p, int enable) {
  if (!p) return SVH_EINVAL;
  p->use_graphs = enable != 0;
  return SVH_OK;
}

}  // extern "C"
