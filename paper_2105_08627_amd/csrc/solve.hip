// Port solve of the saddle system (eq. 7) on the device, FP64.
//
//   K [I; Phi_F] = [A_D^T Phi_D; 0],  K = [[Z, -A_F^T], [A_F, 0]]
//
// Right-preconditioned flexible GMRES (restart m, Sec. III settings), all
// port excitations in lockstep.  The preconditioner is the sparse saddle
// matrix of eq. 12 with Y = |diag Z|, applied through its Schur complement
// (eqs. 13-15): e = d - A Y^-1 c, S b = e with S = A Y^-1 A^T (real, SPD on
// the free nodes), a = Y^-1 (c + A^T b).  S b = e is solved by conjugate
// gradients on the device, preconditioned by an aggregation multigrid (or
// Jacobi), in FP64 (FP32 in the inner solves of the refinement); since that
// inner solve is inexact the outer method is the flexible variant.
// Gram-Schmidt runs twice (CGS2) with all inner products in FP64; the
// Hessenberg columns, Givens rotations and back substitution stay on the
// device, so an Arnoldi step needs no host synchronisation and is replayed
// from a captured graph; the host reads the residual estimates every few
// steps.
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
// The Schur solve works on complex vectors of element type V: double2 in FP64
// solves, float2 in the inner solves of the refinement (their preconditioner
// only has to be approximate); the sparse values stay FP64 and each product
// is rounded to V.
__device__ __forceinline__ float2 vadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 vadd(double2 a, double2 b) { return zadd(a, b); }
__device__ __forceinline__ float2 vsub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 vsub(double2 a, double2 b) { return zsub(a, b); }
__device__ __forceinline__ float2 vscale(float2 a, double s) {
  const float f = (float)s;
  return make_float2(a.x * f, a.y * f);
}
__device__ __forceinline__ double2 vscale(double2 a, double s) { return zscale(a, s); }
template <class V> __device__ __forceinline__ V vzero();
template <> __device__ __forceinline__ float2 vzero<float2>() { return make_float2(0.f, 0.f); }
template <> __device__ __forceinline__ double2 vzero<double2>() { return make_double2(0.0, 0.0); }
template <class V> __device__ __forceinline__ V vfrom(double2 a);
template <> __device__ __forceinline__ float2 vfrom<float2>(double2 a) { return make_float2((float)a.x, (float)a.y); }
template <> __device__ __forceinline__ double2 vfrom<double2>(double2 a) { return a; }
__device__ __forceinline__ double2 vto2(float2 a) { return make_double2(a.x, a.y); }
__device__ __forceinline__ double2 vto2(double2 a) { return a; }

// Work of a conjugate-gradient step is skipped once every right-hand side
// has reached its tolerance (*skip set by k_pcg_start / k_pcg_beta), so a
// fixed number of steps can be enqueued (and replayed from a graph) with only
// the steps that are needed doing work.
#define SKIP_IF_DONE(skip) \
  if ((skip) && *(skip)) return

// e = d - A Y^-1 c (free rows; transpose: d + A Y^-1 c), into node vector e
template <class V>
__global__ void k_pre_rhs(int nrhs, long long N, int CK, int M, const int* __restrict__ rptr,
                          const int* __restrict__ rcol, const double* __restrict__ rval,
                          const uint8_t* __restrict__ freem, const double* __restrict__ ydiag,
                          const double2* __restrict__ in, V* __restrict__ e, int transpose) {
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
    e[r * M + m] = vfrom<V>(acc);
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
template <int SGN, class V>
__device__ __forceinline__ void row_gather(int q0, int q1, const int* __restrict__ c, const double* __restrict__ a,
                                           const V* __restrict__ x, const long long* off, V* acc) {
  int q = q0;
  for (; q + 4 <= q1; q += 4) {
    const int c0 = c[q], c1 = c[q + 1], c2 = c[q + 2], c3 = c[q + 3];
    const double a0 = SGN * a[q], a1 = SGN * a[q + 1], a2 = SGN * a[q + 2], a3 = SGN * a[q + 3];
#pragma unroll
    for (int j = 0; j < kRowRhs; ++j) {
      const V x0 = x[off[j] + c0], x1 = x[off[j] + c1], x2 = x[off[j] + c2], x3 = x[off[j] + c3];
      acc[j] = vadd(acc[j], vscale(x0, a0));
      acc[j] = vadd(acc[j], vscale(x1, a1));
      acc[j] = vadd(acc[j], vscale(x2, a2));
      acc[j] = vadd(acc[j], vscale(x3, a3));
    }
  }
  for (; q < q1; ++q) {
    const int cq = c[q];
    const double aq = SGN * a[q];
#pragma unroll
    for (int j = 0; j < kRowRhs; ++j) acc[j] = vadd(acc[j], vscale(x[off[j] + cq], aq));
  }
}

// u = Y^-1 A^T v (basis-sized), v a node vector with zero Dirichlet entries
template <class V>
__global__ void k_s_half(int nrhs, int CK, int M, const int* __restrict__ cptr, const int* __restrict__ crow,
                         const double* __restrict__ cval, const double* __restrict__ ydiag,
                         const V* __restrict__ v, V* __restrict__ u, const int* __restrict__ skip) {
  SKIP_IF_DONE(skip);
  const int nchunk = (nrhs + kRowRhs - 1) / kRowRhs;
  GRID_STRIDE(i, (long long)CK * nchunk) {
    const int b = (int)(i % CK);
    const int r0 = (int)(i / CK) * kRowRhs;
    const int last = nrhs - 1 - r0;  // >= 0
    long long off[kRowRhs];
    V acc[kRowRhs];
#pragma unroll
    for (int j = 0; j < kRowRhs; ++j) {
      off[j] = (long long)(r0 + min(j, last)) * M;
      acc[j] = vzero<V>();
    }
    row_gather<1>(cptr[b], cptr[b + 1], crow, cval, v, off, acc);
    const double yi = 1.0 / ydiag[b];
#pragma unroll
    for (int j = 0; j < kRowRhs; ++j)
      if (j <= last) u[(long long)(r0 + j) * CK + b] = vscale(acc[j], yi);
  }
}

// q = A u on free nodes (S v = A Y^-1 A^T v)
template <class V>
__global__ void k_s_full(int nrhs, int CK, int M, const int* __restrict__ rptr, const int* __restrict__ rcol,
                         const double* __restrict__ rval, const uint8_t* __restrict__ freem,
                         const V* __restrict__ u, V* __restrict__ q, const int* __restrict__ skip) {
  SKIP_IF_DONE(skip);
  const int nchunk = (nrhs + kRowRhs - 1) / kRowRhs;
  GRID_STRIDE(i, (long long)M * nchunk) {
    const int m = (int)(i % M);
    const int r0 = (int)(i / M) * kRowRhs;
    const int last = nrhs - 1 - r0;  // >= 0
    long long off[kRowRhs];
    V acc[kRowRhs];
#pragma unroll
    for (int j = 0; j < kRowRhs; ++j) {
      off[j] = (long long)(r0 + min(j, last)) * CK;
      acc[j] = vzero<V>();
    }
    if (freem[m]) row_gather<1>(rptr[m], rptr[m + 1], rcol, rval, u, off, acc);
#pragma unroll
    for (int j = 0; j < kRowRhs; ++j)
      if (j <= last) q[(long long)(r0 + j) * M + m] = acc[j];
  }
}

// a = Y^-1 (c + A^T b) (transpose: Y^-1 (c - A^T b)); out = [a; b]
template <class V>
__global__ void k_pre_out(int nrhs, long long N, int CK, int M, const int* __restrict__ cptr,
                          const int* __restrict__ crow, const double* __restrict__ cval,
                          const double* __restrict__ ydiag, const double2* __restrict__ in,
                          const V* __restrict__ bsol, double2* __restrict__ out, int transpose) {
  const long long per = (long long)CK + M;
  GRID_STRIDE(i, per * nrhs) {
    const long long r = i / per, idx = i % per;
    const V* br = bsol + r * M;
    if (idx < CK) {
      double2 acc = make_double2(0, 0);
      for (int q = cptr[idx]; q < cptr[idx + 1]; ++q) acc = zadd(acc, zscale(vto2(br[crow[q]]), cval[q]));
      const double2 c = in[r * N + idx];
      out[r * N + idx] = zscale(transpose ? zsub(c, acc) : zadd(c, acc), 1.0 / ydiag[idx]);
    } else {
      out[r * N + idx] = vto2(br[idx - CK]);
    }
  }
}

// ------------------------------------------------------------ reductions --
// part[g][blk] = sum over the block's chunk of conj(X_g) * Y_g (FP64 sums),
// where pair g = (i, r) reads X at X + i * xs_i + r * xs_r and Y at
// Y + r * ys_r.
template <class V>
__global__ void __launch_bounds__(256) k_mdot(long long n, int nrhs, const V* __restrict__ X, long long xs_i,
                                              long long xs_r, const V* __restrict__ Y, long long ys_r,
                                              double2* __restrict__ part, int conj_x, const int* __restrict__ skip) {
  SKIP_IF_DONE(skip);
  __shared__ double2 sh[256];
  const int g = blockIdx.y;
  const int i = g / nrhs, r = g % nrhs;
  const V* xp = X + (long long)i * xs_i + (long long)r * xs_r;
  const V* yp = Y + (long long)r * ys_r;
  double2 acc = make_double2(0, 0);
  for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
    const double2 xv = vto2(xp[k]), yv = vto2(yp[k]);
    acc = zadd(acc, conj_x ? zcmul(xv, yv) : zmul(xv, yv));
  }
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
// Per right-hand side state on the device (one wavefront, nrhs <= 64):
// thr2 = itol^2 rho0 (a side is done once its rho = r^T D^-1 r falls to it),
// ist[0] = every side done (the skip flag), ist[1] = applications that ended
// with a side short of its tolerance, ist[2 + r] = side r done; steps counts
// the conjugate-gradient steps that did work.

// r = e, b = 0, z = D^-1 r, p = z
template <class V>
__global__ void k_pcg_init(long long n, int M, const double* __restrict__ sdiag, const uint8_t* __restrict__ freem,
                           const V* __restrict__ e, V* __restrict__ r, V* __restrict__ z, V* __restrict__ p,
                           V* __restrict__ b) {
  GRID_STRIDE(i, n) {
    const int m = (int)(i % M);
    const V v = e[i];
    r[i] = v;
    const V zz = freem[m] ? vscale(v, 1.0 / sdiag[m]) : vzero<V>();
    z[i] = zz;
    p[i] = zz;
    b[i] = vzero<V>();
  }
}

// thresholds from rho0 and the tolerance itol2 = itol^2 (device scalar)
__global__ void k_pcg_start(int nrhs, const double2* __restrict__ rho, const double* __restrict__ itol2,
                            double* __restrict__ thr2, int* __restrict__ ist) {
  const int r = threadIdx.x;
  const bool done = r >= nrhs || !(rho[r].x > 0);
  if (r < nrhs) {
    thr2[r] = itol2[0] * rho[r].x;
    ist[2 + r] = done ? 1 : 0;
  }
  const unsigned long long open = __ballot(!done);
  if (r == 0) ist[0] = open == 0ull ? 1 : 0;
}

// alpha = rho / Re(p^H q) per right-hand side (0 when done or degenerate)
__global__ void k_pcg_alpha(int nrhs, const double2* __restrict__ rho, const double2* __restrict__ pq,
                            double* __restrict__ alpha, const int* __restrict__ ist) {
  const int r = threadIdx.x;
  if (r < nrhs) alpha[r] = (!ist[2 + r] && pq[r].x > 0 && rho[r].x > 0) ? rho[r].x / pq[r].x : 0.0;
}

// b += alpha p, r -= alpha q, z = D^-1 r
template <class V>
__global__ void k_pcg_update(long long n, int M, const double* __restrict__ sdiag, const uint8_t* __restrict__ freem,
                             const double* __restrict__ alpha, const V* __restrict__ p, const V* __restrict__ q,
                             V* __restrict__ b, V* __restrict__ r, V* __restrict__ z, const int* __restrict__ skip) {
  SKIP_IF_DONE(skip);
  GRID_STRIDE(i, n) {
    const int m = (int)(i % M);
    const double a = alpha[i / M];
    b[i] = vadd(b[i], vscale(p[i], a));
    const V rr = vsub(r[i], vscale(q[i], a));
    r[i] = rr;
    z[i] = freem[m] ? vscale(rr, 1.0 / sdiag[m]) : vzero<V>();
  }
}

// beta = rho_new / rho, rho = rho_new, and the sides that reach their
// threshold are done (beta = 0 for sides already done)
__global__ void k_pcg_beta(int nrhs, double2* __restrict__ rho, const double2* __restrict__ rho_new,
                           double* __restrict__ beta, const double* __restrict__ thr2, int* __restrict__ ist,
                           long long* __restrict__ steps) {
  if (ist[0]) return;
  const int r = threadIdx.x;
  bool done = true;
  if (r < nrhs) {
    done = ist[2 + r] != 0;
    if (!done) {
      beta[r] = rho[r].x > 0 ? rho_new[r].x / rho[r].x : 0.0;
      rho[r] = rho_new[r];
      done = !(rho_new[r].x > thr2[r]);
      if (done) ist[2 + r] = 1;
    } else {
      beta[r] = 0.0;
    }
  }
  const unsigned long long open = __ballot(!done);
  if (r == 0) {
    ist[0] = open == 0ull ? 1 : 0;
    steps[0] += 1;
  }
}

template <class V>
__global__ void k_pcg_dir(long long n, int M, const double* __restrict__ beta, const V* __restrict__ z,
                          V* __restrict__ p, const int* __restrict__ skip) {
  SKIP_IF_DONE(skip);
  GRID_STRIDE(i, n) p[i] = vadd(z[i], vscale(p[i], beta[i / M]));
}

// end of one application: count it if a side is short of its tolerance
__global__ void k_pcg_end(int* __restrict__ ist) {
  if (threadIdx.x == 0 && !ist[0]) ist[1] += 1;
}

// ------------------------------------------------ multigrid V-cycle (S) --
// Batched over right-hand sides: vectors [r][n] of complex values, level
// matrices real CSR.  wdinv = w_i / a_ii with the Jacobi weight w_i = 0.7, or
// 1 on rows without couplings (solved exactly); the coarse correction is
// scaled by kAmgAlpha < 2 (plain aggregation under-corrects), which keeps the
// cycle symmetric positive definite.
constexpr double kAmgOmega = 0.7;
constexpr double kAmgAlpha = 1.8;

template <class V>
__global__ void k_amg_smooth0(int nrhs, int n, const double* __restrict__ wdinv, const V* __restrict__ b,
                              V* __restrict__ x, const int* __restrict__ skip) {
  SKIP_IF_DONE(skip);
  GRID_STRIDE(i, (long long)n * nrhs) x[i] = vscale(b[i], wdinv[i % n]);
}
// r = b - A x, one row for up to kRowRhs right-hand sides per thread.
template <class V>
__global__ void k_amg_resid(int nrhs, int n, const int* __restrict__ rptr, const int* __restrict__ col,
                            const double* __restrict__ val, const V* __restrict__ b, const V* __restrict__ x,
                            V* __restrict__ r, const int* __restrict__ skip) {
  SKIP_IF_DONE(skip);
  const int nchunk = (nrhs + kRowRhs - 1) / kRowRhs;
  GRID_STRIDE(i, (long long)n * nchunk) {
    const int row = (int)(i % n);
    const int r0 = (int)(i / n) * kRowRhs;
    const int last = nrhs - 1 - r0;  // >= 0
    long long off[kRowRhs];
    V acc[kRowRhs];
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
template <class V>
__global__ void k_amg_resid_w(int nrhs, int n, const int* __restrict__ rptr, const int* __restrict__ col,
                              const double* __restrict__ val, const V* __restrict__ b, const V* __restrict__ x,
                              V* __restrict__ r, const int* __restrict__ skip) {
  SKIP_IF_DONE(skip);
  const int lane = threadIdx.x & 63, rl = lane & 15, g = lane >> 4;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long row = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6; row < n; row += nwaves) {
    const int q0 = rptr[row], q1 = rptr[row + 1];
    for (int r0 = 0; r0 < nrhs; r0 += 16) {
      const long long off = (long long)min(r0 + rl, nrhs - 1) * n;
      V acc = vzero<V>();
      for (int q = q0 + g; q < q1; q += 4) acc = vadd(acc, vscale(x[off + col[q]], val[q]));
      acc.x += __shfl_xor(acc.x, 16);
      acc.y += __shfl_xor(acc.y, 16);
      acc.x += __shfl_xor(acc.x, 32);
      acc.y += __shfl_xor(acc.y, 32);
      if (g == 0 && r0 + rl < nrhs) r[off + row] = vsub(b[off + row], acc);
    }
  }
}
constexpr int kWaveRowLevel = 32768;  // levels with fewer rows take a wavefront per row

template <class V>
__global__ void k_amg_jacobi(int nrhs, int n, const double* __restrict__ wdinv, const V* __restrict__ r,
                             V* __restrict__ x, const int* __restrict__ skip) {
  SKIP_IF_DONE(skip);
  GRID_STRIDE(i, (long long)n * nrhs) x[i] = vadd(x[i], vscale(r[i], wdinv[i % n]));
}
// bc[I] = sum of r over the members of aggregate I
template <class V>
__global__ void k_amg_restrict(int nrhs, int nf, int nc, const int* __restrict__ mptr, const int* __restrict__ mem,
                               const V* __restrict__ r, V* __restrict__ bc, const int* __restrict__ skip) {
  SKIP_IF_DONE(skip);
  GRID_STRIDE(i, (long long)nc * nrhs) {
    const long long rf = (i / nc) * nf;
    const int I = (int)(i % nc);
    V acc = vzero<V>();
    for (int k = mptr[I]; k < mptr[I + 1]; ++k) acc = vadd(acc, r[rf + mem[k]]);
    bc[i] = acc;
  }
}
// x += alpha P xc (rows left out of the coarse level have agg < 0)
template <class V>
__global__ void k_amg_prolong(int nrhs, int nf, int nc, const int* __restrict__ agg, const V* __restrict__ xc,
                              V* __restrict__ x, const int* __restrict__ skip) {
  SKIP_IF_DONE(skip);
  GRID_STRIDE(i, (long long)nf * nrhs) {
    const int a = agg[i % nf];
    if (a >= 0) x[i] = vadd(x[i], vscale(xc[(i / nf) * nc + a], kAmgAlpha));
  }
}
// x = Cinv b on the coarsest level (dense, row-major): a wavefront per output
// element, its lanes over the row and the partial sums joined by lane
// exchanges (a thread per element left the few hundred outputs of this level
// waiting on a chain of n loads each)
template <class V>
__global__ void k_amg_coarse(int nrhs, int n, const double* __restrict__ cinv, const V* __restrict__ b,
                             V* __restrict__ x, const int* __restrict__ skip) {
  SKIP_IF_DONE(skip);
  const int lane = threadIdx.x & 63;
  const long long nw = (long long)gridDim.x * (blockDim.x >> 6);
  for (long long o = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); o < (long long)n * nrhs;
       o += nw) {
    const long long base = (o / n) * n;
    const double* row = cinv + (o % n) * n;
    double2 acc = make_double2(0, 0);
    for (int j = lane; j < n; j += 64) acc = zadd(acc, zscale(vto2(b[base + j]), row[j]));
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      acc.x += __shfl_xor(acc.x, m);
      acc.y += __shfl_xor(acc.y, m);
    }
    if (lane == 0) x[o] = vfrom<V>(acc);
  }
}

template <class V>
__global__ void k_vcopy(long long n, const V* __restrict__ a, V* __restrict__ b) {
  GRID_STRIDE(i, n) b[i] = a[i];
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

// ------------------------------------------- Hessenberg / Givens (device) --
// One wavefront, thread r = right-hand side r (nrhs <= 64).  H is stored per
// side as [restart + 1][restart], the rotations as cs [restart] (real) and sn
// [restart] (complex), the rotated right-hand side g as [restart + 1].
__device__ __forceinline__ double zabs(double2 a) { return hypot(a.x, a.y); }
__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 zdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// start of a cycle: g = (||w||, 0, ...), residual estimate ||w||
__global__ void k_givens_init(int nrhs, int restart, const double2* __restrict__ nrm2, double2* __restrict__ g,
                              double* __restrict__ est) {
  const int r = threadIdx.x;
  if (r >= nrhs) return;
  const double b = sqrt(fmax(nrm2[r].x, 0.0));
  double2* gr = g + (long long)r * (restart + 1);
  gr[0] = make_double2(b, 0.0);
  for (int i = 1; i <= restart; ++i) gr[i] = make_double2(0.0, 0.0);
  est[r] = b;
}

// column j from the Gram-Schmidt coefficients h[i * nrhs + r] (i <= j) and
// ||w||^2 (nrm2[r].x): earlier rotations applied, a new rotation zeroing the
// subdiagonal, g rotated; est[r] = |g[j + 1]|, the residual norm estimate.
__global__ void k_givens(int nrhs, int j, int restart, const double2* __restrict__ h,
                         const double2* __restrict__ nrm2, double2* __restrict__ H, double* __restrict__ cs,
                         double2* __restrict__ sn, double2* __restrict__ g, double* __restrict__ est) {
  const int r = threadIdx.x;
  if (r >= nrhs) return;
  double2* Hr = H + (long long)r * (restart + 1) * restart;
  double* csr = cs + (long long)r * restart;
  double2* snr = sn + (long long)r * restart;
  double2* gr = g + (long long)r * (restart + 1);
  for (int i = 0; i <= j; ++i) Hr[i * restart + j] = h[i * nrhs + r];
  const double hj1 = sqrt(fmax(nrm2[r].x, 0.0));
  for (int i = 0; i < j; ++i) {
    const double2 a = Hr[i * restart + j], b = Hr[(i + 1) * restart + j];
    Hr[i * restart + j] = zadd(zscale(a, csr[i]), zmul(snr[i], b));
    Hr[(i + 1) * restart + j] = zsub(zscale(b, csr[i]), zmul(zconj(snr[i]), a));
  }
  const double2 a = Hr[j * restart + j];
  const double aa = zabs(a);
  double c;
  double2 sv, rr;
  if (aa == 0) {
    c = 0;
    sv = make_double2(1.0, 0.0);
    rr = make_double2(hj1, 0.0);
  } else {
    const double rho = hypot(aa, hj1);
    const double2 ph = zscale(a, 1.0 / aa);
    c = aa / rho;
    sv = zscale(ph, hj1 / rho);
    rr = zscale(ph, rho);
  }
  csr[j] = c;
  snr[j] = sv;
  Hr[j * restart + j] = rr;
  const double2 gj = gr[j];
  gr[j] = zscale(gj, c);
  gr[j + 1] = zscale(zmul(zconj(sv), gj), -1.0);
  est[r] = zabs(gr[j + 1]);
}

// y = H^-1 g over the first nj columns (back substitution), coef[i * nrhs + r] = y_i
__global__ void k_backsolve(int nrhs, int nj, int restart, const double2* __restrict__ H,
                            const double2* __restrict__ g, double2* __restrict__ coef) {
  const int r = threadIdx.x;
  if (r >= nrhs) return;
  const double2* Hr = H + (long long)r * (restart + 1) * restart;
  const double2* gr = g + (long long)r * (restart + 1);
  for (int i = nj - 1; i >= 0; --i) {
    double2 acc = gr[i];
    for (int k = i + 1; k < nj; ++k) acc = zsub(acc, zmul(Hr[i * restart + k], coef[k * nrhs + r]));
    const double2 d = Hr[i * restart + i];
    coef[i * nrhs + r] = zabs(d) > 0 ? zdiv(acc, d) : make_double2(0.0, 0.0);
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
template <class V>
void amg_resid(const svh_problem::AmgDev& L, int nr, const V* b, const V* x, V* r, const int* skip, hipStream_t s) {
  if (L.n < kWaveRowLevel)
    hipLaunchKernelGGL(k_amg_resid_w<V>, dim3(nblocks(64LL * L.n)), dim3(256), 0, s, nr, L.n, L.rptr, L.col, L.val, b,
                       x, r, skip);
  else
    hipLaunchKernelGGL(k_amg_resid<V>, dim3(resid_blocks(L.n, nr)), dim3(256), 0, s, nr, L.n, L.rptr, L.col, L.val,
                       b, x, r, skip);
}

constexpr int kDotBlocks = 256;

struct SolveWs {
  double2 *V, *Zk, *W, *Rhs, *E, *R, *Zp, *P, *Q, *Bs, *U, *part, *h, *h2, *nrm, *rho, *rhon, *pq, *D, *Rr;
  float2 *x32, *y32;
  double *alpha, *beta, *thr2, *itol2, *est, *cs;
  double2 *H, *sn, *g;
  int* ist;
  long long* steps;
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
  char* thr2 = take((size_t)nr * sizeof(double));
  char* itol2 = take(sizeof(double));
  char* est = take((size_t)nr * sizeof(double));
  char* cs = take((size_t)nr * restart * sizeof(double));
  char* H = take((size_t)nr * (restart + 1) * restart * z);
  char* sn = take((size_t)nr * restart * z);
  char* g = take((size_t)nr * (restart + 1) * z);
  char* ist = take((size_t)(2 + nr) * sizeof(int));
  char* steps = take(sizeof(long long));
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
    w->pq = (double2*)pq; w->alpha = (double*)alpha; w->beta = (double*)beta; w->thr2 = (double*)thr2;
    w->itol2 = (double*)itol2; w->est = (double*)est; w->cs = (double*)cs; w->H = (double2*)H;
    w->sn = (double2*)sn; w->g = (double2*)g; w->ist = (int*)ist; w->steps = (long long*)steps;
    w->mv = mv; w->mv_bytes = mvb;
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
  int restart = 0;
  bool op32 = false;      // FP32 operator and FP32 Schur CG (refinement inner solves)
  double t0 = 0;          // start of the solve (progress lines)
  // per mode (0: FP64, 1: refinement inner solve): conjugate-gradient steps
  // per preconditioner application (0: not measured yet), the tolerance they
  // were measured for, and the captured Arnoldi steps (one graph per column)
  int msteps[2] = {0, 0};
  double itol[2] = {-1, -1};
  double itol2_host = 0;
  std::vector<hipGraphExec_t> graphs[2];
  int short_seen = 0;     // applications short of their tolerance, as last read
};

void drop_graphs(Ctx& c, int mode) {
  for (hipGraphExec_t& g : c.graphs[mode])
    if (g) (void)hipGraphExecDestroy(g);
  c.graphs[mode].clear();
}

// out = sum over chunks of conj(X_(i,r)) Y_r into dst[(i * nr + r)]
template <class V>
void mdot(Ctx& c, long long n, int ni, const V* X, long long xs_i, long long xs_r, const V* Y, long long ys_r,
          double2* dst, hipStream_t s, const int* skip = nullptr) {
  hipLaunchKernelGGL(k_mdot<V>, dim3(kDotBlocks, ni * c.nr), dim3(256), 0, s, n, c.nr, X, xs_i, xs_r, Y, ys_r,
                     c.w.part, 1, skip);
  hipLaunchKernelGGL(k_psum, dim3(ni * c.nr), dim3(256), 0, s, kDotBlocks, c.w.part, dst);
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
__global__ void k_ist_reset(int n, int* __restrict__ ist, long long* __restrict__ steps) {
  const int i = threadIdx.x;
  if (i < n) ist[i] = 0;
  if (i == 0) steps[0] = 0;
}

// y = K x (batched columns of length N), enqueued on s; the Z block in FP32
// when c.op32
svh_status apply_K(Ctx& c, const double2* x, double2* y, hipStream_t s) {
  svh_problem* p = c.p;
  std::vector<int32_t> fi(c.nr, c.fidx);
  svh_status st;
  if (c.op32) {
    const long long n = (long long)c.CK * c.nr;
    hipLaunchKernelGGL(k_to32, dim3(nblocks(n)), dim3(256), 0, s, c.nr, c.N, c.CK, x, c.w.x32);
    st = matvec_impl(p, SVH_FP32, c.nr, fi.data(), c.w.x32, c.CK, c.w.y32, c.CK, c.w.mv32, c.w.mv32_bytes, s);
    if (st != SVH_OK) return st;
    hipLaunchKernelGGL(k_from32, dim3(nblocks(n)), dim3(256), 0, s, c.nr, c.N, c.CK, c.w.y32, y);
  } else {
    st = matvec_impl(p, SVH_FP64, c.nr, fi.data(), x, c.N, y, c.N, c.w.mv, c.w.mv_bytes, s);
    if (st != SVH_OK) return st;
  }
  hipLaunchKernelGGL(k_saddle_fix, dim3(nblocks((c.CK + c.M) * (long long)c.nr)), dim3(256), 0, s, c.nr, c.N,
                     c.CK, c.M, p->d_cptr, p->d_crow, p->d_cval, p->d_rptr, p->d_rcol, p->d_rval, p->d_free, x, y,
                     c.transpose);
  SCHK(hipGetLastError());
  return SVH_OK;
}
svh_status apply_K(Ctx& c, const double2* x, double2* y) { return apply_K(c, x, y, c.s); }

template <class V>
void vcycle(Ctx& c, const V* b0, V* x0, const int* skip, hipStream_t s);

// One conjugate-gradient step on S b = e for every right-hand side, enqueued
// on s; a step that finds every side done does no work.
template <class V>
void pcg_step(Ctx& c, hipStream_t s) {
  svh_problem* p = c.p;
  const long long nM = (long long)c.M * c.nr;
  const int* sk = c.w.ist;
  V *P = (V*)c.w.P, *U = (V*)c.w.U, *Q = (V*)c.w.Q, *Bs = (V*)c.w.Bs, *R = (V*)c.w.R, *Zp = (V*)c.w.Zp;
  hipLaunchKernelGGL(k_s_half<V>, dim3(resid_blocks(c.CK, c.nr)), dim3(256), 0, s, c.nr, c.CK, c.M, p->d_cptr,
                     p->d_crow, p->d_cval, p->d_ydiag, P, U, sk);
  hipLaunchKernelGGL(k_s_full<V>, dim3(resid_blocks(c.M, c.nr)), dim3(256), 0, s, c.nr, c.CK, c.M, p->d_rptr,
                     p->d_rcol, p->d_rval, p->d_free, U, Q, sk);
  mdot<V>(c, c.M, 1, P, 0, c.M, Q, c.M, c.w.pq, s, sk);
  hipLaunchKernelGGL(k_pcg_alpha, dim3(1), dim3(64), 0, s, c.nr, c.w.rho, c.w.pq, c.w.alpha, c.w.ist);
  hipLaunchKernelGGL(k_pcg_update<V>, dim3(nblocks(nM)), dim3(256), 0, s, nM, c.M, p->d_sdiag, p->d_free, c.w.alpha,
                     P, Q, Bs, R, Zp, sk);
  if (!p->amg.empty()) vcycle<V>(c, R, Zp, sk, s);
  mdot<V>(c, c.M, 1, R, 0, c.M, Zp, c.M, c.w.rhon, s, sk);
  hipLaunchKernelGGL(k_pcg_beta, dim3(1), dim3(64), 0, s, c.nr, c.w.rho, c.w.rhon, c.w.beta, c.w.thr2, c.w.ist,
                     c.w.steps);
  hipLaunchKernelGGL(k_pcg_dir<V>, dim3(nblocks(nM)), dim3(256), 0, s, nM, c.M, c.w.beta, Zp, P, sk);
}

// out = P in (eqs. 12-15): e from in, S b = e by conjugate gradients to the
// relative tolerance on the device (itol2), a and b to out.  m >= 0: exactly
// m steps are enqueued (the steps after every side is done do no work), with
// no host synchronisation; m < 0: steps in blocks of 8 until the device
// reports every side done or -m steps ran (synchronises; *used = steps run).
template <class V>
svh_status apply_P(Ctx& c, const double2* in, double2* out, int m, hipStream_t s, int* used = nullptr) {
  svh_problem* p = c.p;
  const long long nM = (long long)c.M * c.nr;
  V *E = (V*)c.w.E, *R = (V*)c.w.R, *Zp = (V*)c.w.Zp, *P = (V*)c.w.P, *Bs = (V*)c.w.Bs;
  hipLaunchKernelGGL(k_pre_rhs<V>, dim3(nblocks(nM)), dim3(256), 0, s, c.nr, c.N, c.CK, c.M, p->d_rptr, p->d_rcol,
                     p->d_rval, p->d_free, p->d_ydiag, in, E, c.transpose);
  hipLaunchKernelGGL(k_pcg_init<V>, dim3(nblocks(nM)), dim3(256), 0, s, nM, c.M, p->d_sdiag, p->d_free, E, R, Zp, P,
                     Bs);
  if (!p->amg.empty()) {
    vcycle<V>(c, R, Zp, nullptr, s);
    hipLaunchKernelGGL(k_vcopy<V>, dim3(nblocks(nM)), dim3(256), 0, s, nM, Zp, P);
  }
  mdot<V>(c, c.M, 1, R, 0, c.M, Zp, c.M, c.w.rho, s);
  hipLaunchKernelGGL(k_pcg_start, dim3(1), dim3(64), 0, s, c.nr, c.w.rho, c.w.itol2, c.w.thr2, c.w.ist);
  if (m >= 0) {
    for (int k = 0; k < m; ++k) pcg_step<V>(c, s);
  } else {
    int done = 0, k = 0;
    while (k < -m) {
      for (int q = 0; q < 8; ++q) pcg_step<V>(c, s);
      k += 8;
      SCHK(hipMemcpyAsync(&done, c.w.ist, sizeof(int), hipMemcpyDeviceToHost, s));
      SCHK(hipStreamSynchronize(s));
      if (done) break;
    }
    if (used) *used = k;
  }
  hipLaunchKernelGGL(k_pcg_end, dim3(1), dim3(64), 0, s, c.w.ist);
  hipLaunchKernelGGL(k_pre_out<V>, dim3(nblocks((c.CK + c.M) * (long long)c.nr)), dim3(256), 0, s, c.nr, c.N, c.CK,
                     c.M, p->d_cptr, p->d_crow, p->d_cval, p->d_ydiag, in, Bs, out, c.transpose);
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
// side.  Level vectors are used as V arrays (FP32 ones fit in the FP64
// allocation).
template <class V>
void vcycle(Ctx& c, const V* b0, V* x0, const int* skip, hipStream_t s) {
  svh_problem* p = c.p;
  const int nl = (int)p->amg.size(), nr = c.nr;
  for (int l = 0; l < nl; ++l) {
    auto& L = p->amg[l];
    const V* b = l ? (const V*)L.b : b0;
    V* x = l ? (V*)L.x : x0;
    V* r = (V*)L.r;
    const long long n = (long long)L.n * nr;
    if (l == nl - 1) {
      if (p->amg_coarse == kAmgCoarseDense) {
        hipLaunchKernelGGL(k_amg_coarse<V>, dim3(nblocks(64 * n)), dim3(256), 0, s, nr, L.n, p->d_amg_cinv, b, x, skip);
      } else {  // diagonal matrix (exact), or damped Jacobi sweeps
        hipLaunchKernelGGL(k_amg_smooth0<V>, dim3(nblocks(n)), dim3(256), 0, s, nr, L.n, L.dinv, b, x, skip);
        for (int k = 1; k < (p->amg_coarse == kAmgCoarseJacobi ? kAmgCoarseSweeps : 1); ++k) {
          amg_resid<V>(L, nr, b, x, r, skip, s);
          hipLaunchKernelGGL(k_amg_jacobi<V>, dim3(nblocks(n)), dim3(256), 0, s, nr, L.n, L.dinv, r, x, skip);
        }
      }
      break;
    }
    hipLaunchKernelGGL(k_amg_smooth0<V>, dim3(nblocks(n)), dim3(256), 0, s, nr, L.n, L.dinv, b, x, skip);
    amg_resid<V>(L, nr, b, x, r, skip, s);
    auto& Cl = p->amg[l + 1];
    hipLaunchKernelGGL(k_amg_restrict<V>, dim3(nblocks((long long)Cl.n * nr)), dim3(256), 0, s, nr, L.n, Cl.n,
                       L.mptr, L.mem, r, (V*)Cl.b, skip);
  }
  for (int l = nl - 2; l >= 0; --l) {
    auto& L = p->amg[l];
    auto& Cl = p->amg[l + 1];
    const V* b = l ? (const V*)L.b : b0;
    V* x = l ? (V*)L.x : x0;
    V* r = (V*)L.r;
    const long long n = (long long)L.n * nr;
    hipLaunchKernelGGL(k_amg_prolong<V>, dim3(nblocks(n)), dim3(256), 0, s, nr, L.n, Cl.n, L.agg, (const V*)Cl.x, x,
                       skip);
    amg_resid<V>(L, nr, b, x, r, skip, s);
    hipLaunchKernelGGL(k_amg_jacobi<V>, dim3(nblocks(n)), dim3(256), 0, s, nr, L.n, L.dinv, r, x, skip);
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

struct FgmresStats {
  int total = 0, inner = 0, restarts = 0;
};

svh_status finish(Ctx& c, svh_status st) {
  drop_graphs(c, 0);
  drop_graphs(c, 1);
  return st;
}

// per-column 2-norms of a batch of N-vectors
svh_status norms(Ctx& c, const double2* v, std::vector<double>& out) {
  svh_problem* p = c.p;
  mdot<double2>(c, c.N, 1, v, 0, c.N, v, c.N, c.w.nrm, c.s);
  std::vector<double2> h(c.nr);
  SCHK(hipMemcpyAsync(h.data(), c.w.nrm, sizeof(double2) * c.nr, hipMemcpyDeviceToHost, c.s));
  SCHK(hipStreamSynchronize(c.s));
  out.resize(c.nr);
  for (int r = 0; r < c.nr; ++r) out[r] = std::sqrt(std::max(h[r].x, 0.0));
  return SVH_OK;
}

constexpr int kInnerMax = 20000;  // conjugate-gradient steps per application at most
// default Schur CG tolerance of the refinement's inner solves, whose CG runs
// in FP32 (about 1e-7 of rounding); the preconditioner of a flexible GMRES
// need not be exact
constexpr double kIrSchurTol = 1e-4;
// Arnoldi steps between reads of the residual estimates, and every step once
// the worst estimate is within kCheckNear of its target
constexpr int kCheckEvery = 4;
constexpr double kCheckNear = 30.0;

// One Arnoldi step of column j, enqueued on s without host synchronisation
// (unless probe != nullptr): Zk_j = P V_j with m inner steps, w = K Zk_j,
// CGS2 against V_0..V_j, V_{j+1} = w / ||w||, and the Hessenberg column
// rotated on the device (est = residual estimates).  probe: the inner solve
// runs to its tolerance with host checks and *probe receives its steps.
svh_status arnoldi_step(Ctx& c, int j, int m, hipStream_t s, int* probe = nullptr) {
  svh_problem* p = c.p;
  const int nr = c.nr;
  const long long NN = c.N * nr, vs = NN;
  svh_status st = c.op32 ? apply_P<float2>(c, c.w.V + j * vs, c.w.Zk + j * vs, probe ? -kInnerMax : m, s, probe)
                         : apply_P<double2>(c, c.w.V + j * vs, c.w.Zk + j * vs, probe ? -kInnerMax : m, s, probe);
  if (st != SVH_OK) return st;
  if ((st = apply_K(c, c.w.Zk + j * vs, c.w.W, s)) != SVH_OK) return st;
  mdot<double2>(c, c.N, j + 1, c.w.V, vs, c.N, c.w.W, c.N, c.w.h, s);
  hipLaunchKernelGGL(k_cgs_update, dim3(nblocks(NN)), dim3(256), 0, s, c.N, nr, j + 1, c.w.V, vs, c.w.h, c.w.W);
  mdot<double2>(c, c.N, j + 1, c.w.V, vs, c.N, c.w.W, c.N, c.w.h2, s);
  hipLaunchKernelGGL(k_cgs_update, dim3(nblocks(NN)), dim3(256), 0, s, c.N, nr, j + 1, c.w.V, vs, c.w.h2, c.w.W);
  hipLaunchKernelGGL(k_add_small, dim3(((j + 1) * nr + 255) / 256), dim3(256), 0, s, (j + 1) * nr, c.w.h, c.w.h2);
  mdot<double2>(c, c.N, 1, c.w.W, 0, c.N, c.w.W, c.N, c.w.nrm, s);
  hipLaunchKernelGGL(k_normalize, dim3(nblocks(NN)), dim3(256), 0, s, c.N, nr, c.w.nrm, c.w.W, c.w.V + (j + 1) * vs);
  hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, s, nr, j, c.restart, c.w.h, c.w.nrm, c.w.H, c.w.cs, c.w.sn,
                     c.w.g, c.w.est);
  SCHK(hipGetLastError());
  return SVH_OK;
}

// The Arnoldi step of column j replayed from a graph captured on the
// problem's private stream (all operands are fixed workspace buffers, so one
// graph per column serves every cycle of the solve).
svh_status graph_step(Ctx& c, int j) {
  svh_problem* p = c.p;
  const int mode = c.op32 ? 1 : 0;
  std::vector<hipGraphExec_t>& gv = c.graphs[mode];
  if ((int)gv.size() < c.restart) gv.resize(c.restart, nullptr);
  if (!gv[j]) {
    if (!p->cap_stream) SCHK(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    SCHK(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    const svh_status st = arnoldi_step(c, j, c.msteps[mode], p->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
    if (st != SVH_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    SCHK(e);
    const hipError_t ei = hipGraphInstantiate(&gv[j], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    SCHK(ei);
  }
  SCHK(hipGraphLaunch(gv[j], c.s));
  return SVH_OK;
}

// Right-preconditioned flexible GMRES(restart) on K X = B for every column,
// starting from the X given; stops when every column's residual estimate is
// below rre * bnorm[r] or after maxit steps.  The inner solve runs to the
// relative tolerance itol: its step count per application is measured once
// (with host checks), then every Arnoldi step is enqueued (or replayed from
// its graph) without host synchronisation, and the residual estimates are
// read every kCheckEvery steps.  When an application ends short of itol, the
// step count doubles (up to kInnerMax) and the graphs are captured again.
svh_status fgmres(Ctx& c, const double2* B, double2* X, const std::vector<double>& bnorm, double rre, int restart,
                  int maxit, double itol, FgmresStats& fs, int max_cycles = 1 << 30) {
  svh_problem* p = c.p;
  const int nr = c.nr;
  const int mode = c.op32 ? 1 : 0;
  const long long NN = c.N * nr;
  const long long vs = NN;  // stride between Krylov vectors
  const bool graphs = p->use_graphs && !p->prof;
  svh_status st;
  if (itol != c.itol[mode]) {
    c.itol[mode] = itol;
    c.msteps[mode] = 0;
    drop_graphs(c, mode);
  }
  c.itol2_host = itol * itol;
  SCHK(hipMemcpyAsync(c.w.itol2, &c.itol2_host, sizeof(double), hipMemcpyHostToDevice, c.s));
  int steps = 0, cycles = 0;
  bool first = true;
  std::vector<double> est(nr, 0.0);
  int hist[2] = {0, 0};
  long long inner = 0;
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
    hipLaunchKernelGGL(k_givens_init, dim3(1), dim3(64), 0, c.s, nr, restart, c.w.nrm, c.w.g, c.w.est);
    int jdone = 0;
    bool near = false;
    for (int j = 0; j < restart && steps < maxit; ++j) {
      if (c.msteps[mode] == 0) {
        int used = 0;
        if ((st = arnoldi_step(c, j, 0, c.s, &used)) != SVH_OK) return st;
        c.msteps[mode] = std::min(kInnerMax, (used + std::max(4, used / 4) + 3) / 4 * 4);
      } else if (graphs) {
        if ((st = graph_step(c, j)) != SVH_OK) return st;
      } else {
        if ((st = arnoldi_step(c, j, c.msteps[mode], c.s)) != SVH_OK) return st;
      }
      ++steps;
      ++fs.total;
      jdone = j + 1;
      if (jdone % kCheckEvery == 0 || near || jdone == restart || steps >= maxit) {
        SCHK(hipMemcpyAsync(est.data(), c.w.est, sizeof(double) * nr, hipMemcpyDeviceToHost, c.s));
        SCHK(hipMemcpyAsync(hist, c.w.ist, sizeof(int) * 2, hipMemcpyDeviceToHost, c.s));
        SCHK(hipMemcpyAsync(&inner, c.w.steps, sizeof(long long), hipMemcpyDeviceToHost, c.s));
        SCHK(hipStreamSynchronize(c.s));
        fs.inner = (int)inner;
        if (hist[1] > c.short_seen) {
          c.short_seen = hist[1];
          if (c.msteps[mode] < kInnerMax) {
            c.msteps[mode] = std::min(kInnerMax, (c.msteps[mode] * 3 / 2 + 3) / 4 * 4);
            drop_graphs(c, mode);
          }
        }
        double worst = 0;
        for (int r = 0; r < nr; ++r)
          if (bnorm[r] > 0) worst = std::max(worst, est[r] / (rre * bnorm[r]));
        if (worst <= 1.0) break;
        near = worst <= kCheckNear;
      }
    }
    // y = H^-1 g, x += Zk y
    hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(64), 0, c.s, nr, jdone, restart, c.w.H, c.w.g, c.w.h2);
    hipLaunchKernelGGL(k_combine, dim3(nblocks(NN)), dim3(256), 0, c.s, c.N, nr, jdone, c.w.Zk, vs, c.w.h2, X);
    SCHK(hipGetLastError());
    ++fs.restarts;
    ++cycles;
    if (verbose(p)) {
      double worst = 0;
      for (int r = 0; r < nr; ++r)
        if (bnorm[r] > 0) worst = std::max(worst, est[r] / bnorm[r]);
      std::fprintf(stderr, "[svh] fgmres cycle %d (%s): %d steps, estimate %.3e, inner CG steps %d (%d per "
                   "application), %.2f s\n", cycles, c.op32 ? "fp32 operator" : "fp64", fs.total, worst, fs.inner,
                   c.msteps[mode], now_s() - c.t0);
      std::fflush(stderr);
    }
  }
  SCHK(hipStreamSynchronize(c.s));
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
  c.restart = restart;
  c.t0 = now_s();
  carve(p, restart, prec, static_cast<char*>((void*)(((uintptr_t)ws + 255) & ~(uintptr_t)255)), &c.w);
  hipLaunchKernelGGL(k_ist_reset, dim3(1), dim3(128), 0, c.s, 2 + c.nr, c.w.ist, c.w.steps);
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
    const double itol = p->schur_tol > 0 ? p->schur_tol : std::max(1e-12, std::min(1e-8, rre));
    st = fgmres(c, c.w.Rhs, X, bnorm, rre, restart, maxit, itol, fs);
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
                  p->schur_tol > 0 ? p->schur_tol : kIrSchurTol, fs, 1);
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
