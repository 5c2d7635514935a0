// Tucker-SVD of the circulant Green spectrum (Algorithm 1, Sec. II.B), host.
//
// The circulant tensor Z = FFT3(E) with E the even circulant embedding of the
// Toeplitz tensor T (Sec. II.A).  Per axis the embedding is E = P T with
// P (L x K) copying offset n to positions n and L - n; P = Q W^(1/2) with Q
// orthonormal and W = diag(1, 2, 2, ...).  The DFT divided by sqrt(L) is
// unitary, so with Tw = T scaled by sqrt(w1 w2 w3) every unfolding of Z is
// (unitary) x (unfolding of Tw) x (unitary): the mode-i singular values of Z
// are sqrt(L1 L2 L3) times those of Tw and its left singular vectors are
// DFT(Q u)/sqrt(L) for the left singular vectors u of Tw, i.e. the real
// cosine series  (u_0 + sqrt(2) sum_{n>=1} u_n cos(2 pi k n / L)) / sqrt(L).
// Algorithm 1 on Z (unfold, SVD, truncate at tol/sqrt(3) per mode, project)
// therefore gives exactly the factors computed here from the K1 x K2 x K3
// tensor Tw instead of the eight times larger L1 x L2 x L3 tensor Z.
//
// An axis on which T is odd (T(-n) = -T(n), so T(0) = 0) embeds as
// E(n) = -T(n), E(L - n) = T(n); its spectrum is j times the sine series
// 2 sum_{n>=1} T_n sin(2 pi k n / L), the weights are w_0 = 0, w_n = 2 and the
// factor columns are  sqrt(2) sum_{n>=1} u_n sin(2 pi k n / L) / sqrt(L).  The
// stored factors are real; the caller keeps track of the factor j per odd axis.
//
// Each mode's SVD: Householder QR of the transposed unfolding, then one-sided
// (Hestenes) Jacobi on the triangular factor, which keeps small singular
// values accurate relative to the largest one (no Gram matrix is formed).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "host_math.h"

namespace svh {

// Householder QR of A (m x n, column-major, m >= n); returns R (n x n,
// column-major, upper triangular).
static void householder_r(std::vector<double>& A, int m, int n, std::vector<double>& R) {
  std::vector<double> v(m);
  for (int j = 0; j < n; ++j) {
    double* aj = &A[(size_t)j * m];
    double nrm2 = 0;
    for (int i = j; i < m; ++i) nrm2 += aj[i] * aj[i];
    const double nrm = std::sqrt(nrm2);
    if (nrm == 0) continue;
    const double alpha = aj[j] > 0 ? -nrm : nrm;
    for (int i = j; i < m; ++i) v[i] = aj[i];
    v[j] -= alpha;
    const double vv = nrm2 - aj[j] * aj[j] + v[j] * v[j];
    aj[j] = alpha;
    for (int i = j + 1; i < m; ++i) aj[i] = 0;
    if (vv == 0) continue;
    const double beta = 2.0 / vv;
#pragma omp parallel for schedule(static)
    for (int k = j + 1; k < n; ++k) {
      double* ak = &A[(size_t)k * m];
      double s = 0;
      for (int i = j; i < m; ++i) s += v[i] * ak[i];
      s *= beta;
      for (int i = j; i < m; ++i) ak[i] -= s * v[i];
    }
  }
  R.assign((size_t)n * n, 0.0);
  for (int k = 0; k < n; ++k)
    for (int i = 0; i <= k; ++i) R[(size_t)k * n + i] = A[(size_t)k * m + i];
}

// One-sided Jacobi on A (m x n column-major): A V = B with orthogonal columns.
// Returns column norms (singular values) and V (n x n column-major).
static void hestenes(std::vector<double>& A, int m, int n, std::vector<double>& sig,
                     std::vector<double>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  const int np = n + (n & 1);
  std::vector<int> ring(np);
  std::iota(ring.begin(), ring.end(), 0);
  for (int sweep = 0; sweep < 80; ++sweep) {
    double off = 0;
    for (int round = 0; round < np - 1; ++round) {
#pragma omp parallel for schedule(dynamic, 1) reduction(max : off)
      for (int t = 0; t < np / 2; ++t) {
        int p = ring[t], q = ring[np - 1 - t];
        if (p >= n || q >= n) continue;
        if (p > q) std::swap(p, q);
        double* ap = &A[(size_t)p * m];
        double* aq = &A[(size_t)q * m];
        double al = 0, be = 0, ga = 0;
        for (int i = 0; i < m; ++i) {
          al += ap[i] * ap[i];
          be += aq[i] * aq[i];
          ga += ap[i] * aq[i];
        }
        if (al < 1e-300 || be < 1e-300) continue;
        const double rel = std::fabs(ga) / std::sqrt(al * be);
        if (rel <= 1e-15) continue;
        off = std::max(off, rel);
        const double zeta = (be - al) / (2 * ga);
        const double tt = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1 + zeta * zeta));
        const double c = 1 / std::sqrt(1 + tt * tt), s = c * tt;
        for (int i = 0; i < m; ++i) {
          const double x = ap[i], y = aq[i];
          ap[i] = c * x - s * y;
          aq[i] = s * x + c * y;
        }
        double* vp = &V[(size_t)p * n];
        double* vq = &V[(size_t)q * n];
        for (int i = 0; i < n; ++i) {
          const double x = vp[i], y = vq[i];
          vp[i] = c * x - s * y;
          vq[i] = s * x + c * y;
        }
      }
      // rotate the tournament ring (first element fixed)
      const int last = ring[np - 1];
      for (int i = np - 1; i > 1; --i) ring[i] = ring[i - 1];
      ring[1] = last;
    }
    if (off <= 1e-15) break;
  }
  sig.resize(n);
  for (int j = 0; j < n; ++j) {
    double s = 0;
    for (int i = 0; i < m; ++i) s += A[(size_t)j * m + i] * A[(size_t)j * m + i];
    sig[j] = std::sqrt(s);
  }
}

// Left singular vectors (K x r, row-major U[k*r + c], sorted by decreasing
// singular value) and singular values of the mode-`mode` unfolding of X.
static void mode_svd(const std::vector<double>& X, const int K[3], int mode,
                     std::vector<double>& U, std::vector<double>& sig, int& r) {
  const int Km = K[mode];
  const size_t P = (size_t)K[0] * K[1] * K[2] / Km;
  // Mt: P x Km column-major; column j = all entries whose mode index is j
  std::vector<double> Mt(P * Km);
  for (int k = 0; k < K[2]; ++k)
    for (int j = 0; j < K[1]; ++j)
      for (int i = 0; i < K[0]; ++i) {
        const int idx[3] = {i, j, k};
        const int o0 = (mode + 1) % 3, o1 = (mode + 2) % 3;
        const size_t row = (size_t)idx[o0] + (size_t)K[o0] * idx[o1];
        Mt[(size_t)idx[mode] * P + row] = X[((size_t)k * K[1] + j) * K[0] + i];
      }
  std::vector<double> vecs;  // Km x r column-major
  std::vector<double> s;
  if (P >= (size_t)Km) {
    std::vector<double> R;
    householder_r(Mt, (int)P, Km, R);
    std::vector<double> V;
    hestenes(R, Km, Km, s, V);  // left singular vectors of M = columns of V
    r = Km;
    vecs = V;
  } else {
    // M (Km x P, tall): Hestenes directly; U = B / sigma
    std::vector<double> M((size_t)Km * P);
    for (size_t p = 0; p < P; ++p)
      for (int j = 0; j < Km; ++j) M[p * Km + j] = Mt[(size_t)j * P + p];
    std::vector<double> V;
    hestenes(M, Km, (int)P, s, V);
    r = (int)P;
    vecs.assign((size_t)Km * r, 0.0);
    for (int c = 0; c < r; ++c)
      for (int j = 0; j < Km; ++j)
        vecs[(size_t)c * Km + j] = s[c] > 0 ? M[(size_t)c * Km + j] / s[c] : 0.0;
  }
  std::vector<int> order(r);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return s[a] > s[b]; });
  U.assign((size_t)Km * r, 0.0);
  sig.resize(r);
  for (int c = 0; c < r; ++c) {
    sig[c] = s[order[c]];
    for (int j = 0; j < Km; ++j) U[(size_t)j * r + c] = vecs[(size_t)order[c] * Km + j];
  }
}

// Smallest d with sqrt(sum_{j>=d} sig_j^2) <= thr (d >= 1).
static int select_rank(const std::vector<double>& sig, double thr, double& tail_out) {
  const int r = (int)sig.size();
  std::vector<double> tail(r + 1, 0.0);
  for (int j = r - 1; j >= 0; --j) tail[j] = tail[j + 1] + sig[j] * sig[j];
  int d = r;
  for (int j = 0; j <= r; ++j)
    if (std::sqrt(tail[j]) <= thr) { d = j; break; }
  d = std::max(d, 1);
  tail_out = std::sqrt(tail[d]);
  return d;
}

static double cos2pi_frac(long long num, long long den) {
  // cos(2 pi num / den) with exact reduction of the integer argument
  long long m = num % den;
  if (m < 0) m += den;
  const long double a = 2.0L * 3.141592653589793238462643383279502884L * (long double)m / (long double)den;
  return (double)cosl(a);
}

static double sin2pi_frac(long long num, long long den) {
  long long m = num % den;
  if (m < 0) m += den;
  const long double a = 2.0L * 3.141592653589793238462643383279502884L * (long double)m / (long double)den;
  return (double)sinl(a);
}

// Tucker factors of the spectrum of the circulant embedding of T (T:
// [K3][K2][K1], x fastest; L: FFT lengths, L[i] >= 2 K[i] - 1; odd[i] != 0
// where T is odd along axis i).
int tucker_circulant(const int K[3], const int L[3], const double* T, const int odd[3], double tol,
                     TuckerFactors& out) {
  const size_t n = (size_t)K[0] * K[1] * K[2];
  std::vector<double> Tw(n);
  const double r2 = std::sqrt(2.0);
  double nrm2 = 0;
  for (int k = 0; k < K[2]; ++k)
    for (int j = 0; j < K[1]; ++j)
      for (int i = 0; i < K[0]; ++i) {
        const int idx[3] = {i, j, k};
        double w = 1.0;
        for (int a = 0; a < 3; ++a) w *= idx[a] ? r2 : (odd[a] ? 0.0 : 1.0);
        const size_t b = ((size_t)k * K[1] + j) * K[0] + i;
        Tw[b] = T[b] * w;
        nrm2 += Tw[b] * Tw[b];
      }
  const double nrm = std::sqrt(nrm2);
  if (!(nrm > 0)) {
    // zero tensor (an odd family on a grid one voxel wide along its axis):
    // rank one with zero factors
    for (int m = 0; m < 3; ++m) {
      out.d[m] = 1;
      out.F[m].assign((size_t)L[m], 0.0);
    }
    out.core.assign(1, 0.0);
    out.relerr = 0;
    return 1;
  }
  const double thr = tol / std::sqrt(3.0) * nrm;
  std::vector<double> U[3];
  double tails2 = 0;
  for (int m = 0; m < 3; ++m) {
    std::vector<double> sig, Ufull;
    int r = 0;
    mode_svd(Tw, K, m, Ufull, sig, r);
    double tail = 0;
    const int d = select_rank(sig, thr, tail);
    tails2 += tail * tail;
    out.d[m] = d;
    U[m].resize((size_t)K[m] * d);
    for (int j = 0; j < K[m]; ++j)
      for (int c = 0; c < d; ++c) U[m][(size_t)j * d + c] = Ufull[(size_t)j * r + c];
  }
  out.relerr = std::sqrt(tails2) / nrm;
  const int d1 = out.d[0], d2 = out.d[1], d3 = out.d[2];
  // core = Tw x1 U1^T x2 U2^T x3 U3^T
  std::vector<double> G1((size_t)K[2] * K[1] * d1, 0.0);
#pragma omp parallel for collapse(2)
  for (int k = 0; k < K[2]; ++k)
    for (int j = 0; j < K[1]; ++j)
      for (int a = 0; a < d1; ++a) {
        double s = 0;
        const double* t = &Tw[((size_t)k * K[1] + j) * K[0]];
        for (int i = 0; i < K[0]; ++i) s += U[0][(size_t)i * d1 + a] * t[i];
        G1[((size_t)k * K[1] + j) * d1 + a] = s;
      }
  std::vector<double> G2((size_t)K[2] * d2 * d1, 0.0);
#pragma omp parallel for collapse(2)
  for (int k = 0; k < K[2]; ++k)
    for (int b = 0; b < d2; ++b)
      for (int a = 0; a < d1; ++a) {
        double s = 0;
        for (int j = 0; j < K[1]; ++j) s += U[1][(size_t)j * d2 + b] * G1[((size_t)k * K[1] + j) * d1 + a];
        G2[((size_t)k * d2 + b) * d1 + a] = s;
      }
  const double scale = std::sqrt((double)L[0]) * std::sqrt((double)L[1]) * std::sqrt((double)L[2]);
  out.core.assign((size_t)d3 * d2 * d1, 0.0);
#pragma omp parallel for collapse(2)
  for (int c = 0; c < d3; ++c)
    for (int b = 0; b < d2; ++b)
      for (int a = 0; a < d1; ++a) {
        double s = 0;
        for (int k = 0; k < K[2]; ++k) s += U[2][(size_t)k * d3 + c] * G2[((size_t)k * d2 + b) * d1 + a];
        out.core[((size_t)c * d2 + b) * d1 + a] = s * scale;
      }
  // circulant factors: cosine (even axis) or sine (odd axis) series of the
  // Toeplitz factors
  for (int m = 0; m < 3; ++m) {
    const int d = out.d[m];
    out.F[m].assign((size_t)L[m] * d, 0.0);
    const double inv = 1.0 / std::sqrt((double)L[m]);
    const bool od = odd[m] != 0;
#pragma omp parallel for
    for (int k = 0; k < L[m]; ++k)
      for (int c = 0; c < d; ++c) {
        double s = od ? 0.0 : U[m][c];
        for (int j = 1; j < K[m]; ++j)
          s += r2 * U[m][(size_t)j * d + c] *
               (od ? sin2pi_frac((long long)k * j, L[m]) : cos2pi_frac((long long)k * j, L[m]));
        out.F[m][(size_t)k * d + c] = s * inv;
      }
  }
  return 0;
}

// Tucker-SVD (Algorithm 1) of T itself: F[i] = leading left singular vectors
// of the mode-i unfolding (K_i x d_i, [k][c]), core = T x1 F1^T x2 F2^T x3 F3^T.
int tucker_plain(const int K[3], const double* T, double tol, TuckerFactors& out) {
  const size_t n = (size_t)K[0] * K[1] * K[2];
  std::vector<double> X(T, T + n);
  double nrm2 = 0;
  for (size_t i = 0; i < n; ++i) nrm2 += X[i] * X[i];
  const double nrm = std::sqrt(nrm2);
  if (!(nrm > 0)) {
    for (int m = 0; m < 3; ++m) {
      out.d[m] = 1;
      out.F[m].assign((size_t)K[m], 0.0);
    }
    out.core.assign(1, 0.0);
    out.relerr = 0;
    return 1;
  }
  const double thr = tol / std::sqrt(3.0) * nrm;
  double tails2 = 0;
  for (int m = 0; m < 3; ++m) {
    std::vector<double> sig, Ufull;
    int r = 0;
    mode_svd(X, K, m, Ufull, sig, r);
    double tail = 0;
    const int d = select_rank(sig, thr, tail);
    tails2 += tail * tail;
    out.d[m] = d;
    out.F[m].resize((size_t)K[m] * d);
    for (int j = 0; j < K[m]; ++j)
      for (int c = 0; c < d; ++c) out.F[m][(size_t)j * d + c] = Ufull[(size_t)j * r + c];
  }
  out.relerr = std::sqrt(tails2) / nrm;
  const int d1 = out.d[0], d2 = out.d[1], d3 = out.d[2];
  const std::vector<double>&U0 = out.F[0], &U1 = out.F[1], &U2 = out.F[2];
  std::vector<double> G1((size_t)K[2] * K[1] * d1, 0.0);
#pragma omp parallel for collapse(2)
  for (int k = 0; k < K[2]; ++k)
    for (int j = 0; j < K[1]; ++j)
      for (int a = 0; a < d1; ++a) {
        double s = 0;
        const double* t = &X[((size_t)k * K[1] + j) * K[0]];
        for (int i = 0; i < K[0]; ++i) s += U0[(size_t)i * d1 + a] * t[i];
        G1[((size_t)k * K[1] + j) * d1 + a] = s;
      }
  std::vector<double> G2((size_t)K[2] * d2 * d1, 0.0);
#pragma omp parallel for collapse(2)
  for (int k = 0; k < K[2]; ++k)
    for (int b = 0; b < d2; ++b)
      for (int a = 0; a < d1; ++a) {
        double s = 0;
        for (int j = 0; j < K[1]; ++j) s += U1[(size_t)j * d2 + b] * G1[((size_t)k * K[1] + j) * d1 + a];
        G2[((size_t)k * d2 + b) * d1 + a] = s;
      }
  out.core.assign((size_t)d3 * d2 * d1, 0.0);
#pragma omp parallel for collapse(2)
  for (int c = 0; c < d3; ++c)
    for (int b = 0; b < d2; ++b)
      for (int a = 0; a < d1; ++a) {
        double s = 0;
        for (int k = 0; k < K[2]; ++k) s += U2[(size_t)k * d3 + c] * G2[((size_t)k * d2 + b) * d1 + a];
        out.core[((size_t)c * d2 + b) * d1 + a] = s;
      }
  return 0;
}

int tucker_even_circulant(const int K[3], const int L[3], const double* T, double tol, TuckerFactors& out) {
  const int even[3] = {0, 0, 0};
  return tucker_circulant(K, L, T, even, tol, out);
}

}  // namespace svh
