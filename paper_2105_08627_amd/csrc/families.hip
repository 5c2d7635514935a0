// Voxel-pair integral families of the piecewise-linear basis (eqs. 5-8,
// App. A eqs. 20-21), on the device.
//
// For unit voxels with centres d apart (source minus observer), u / u' the
// observer / source points relative to their centres and g = 1/(4 pi |r|):
//   M0   = int int g(d + u' - u)
//   M1_a = int int u'_a g(d + u' - u)        (source moment)
//   M2_a = int int u_a u'_a g(d + u' - u)
// With v = u' - u each becomes a 3D integral over [-1,1]^3 of the product of
// per-axis overlap weights of two unit intervals,
//   (u, u') powers (0,0): 1 - |v|;  (0,1): v (1 - |v|) / 2;
//   (1,1): -t/4 + t^2/2 - t^3/6 with t = 1 - |v|,
// times g(d + v).  The weights are polynomials on [-1,0] and [0,1], so the
// integral splits into 8 boxes.  Offsets with max |d_i| >= 2 keep the
// singular point outside every box: tensor Gauss-Legendre per box with a
// point count from the box's distance to it (this kernel).  The 8 offsets
// with all d_i in {0, 1} are computed on the host by an exact reduction of
// each box's monomial integrals to regular face integrals (below).
#include <cmath>
#include <vector>

#include "svh_internal.h"

namespace svh {

// families in the order M0, M1x, M1y, M1z, M2x, M2y, M2z (kNFam)
// Gauss-Legendre tiers: point count per axis by distance to the singularity
constexpr int kTiers = 5;
constexpr int kTierN[kTiers] = {6, 8, 10, 14, 20};
constexpr double kTierDist[kTiers] = {32.0, 12.0, 5.0, 2.0, 0.0};
constexpr int kTierOff[kTiers] = {0, 6, 14, 24, 38};
constexpr int kGlTotal = 58;

__constant__ double c_glx[kGlTotal];
__constant__ double c_glw[kGlTotal];

// Gauss-Legendre nodes and weights on [0, 1] by Newton iteration on P_n.
static void gauss_legendre01(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    long double z = cosl(3.141592653589793238462643383279502884L * (i + 0.75L) / (n + 0.5L));
    long double dp = 0;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const long double pk = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      dp = n * (z * p1 - p0) / (z * z - 1);
      const long double dz = p1 / dp;
      z -= dz;
      if (fabsl(dz) < 1e-19L) break;
    }
    x[i] = (double)((1 - z) / 2);
    w[i] = (double)(1 / ((1 - z * z) * dp * dp));  // 2/((1-z^2)P'^2) scaled by 1/2
  }
}

__host__ __device__ inline void axis_weights(double v, double& w0, double& w1, double& w2) {
  const double a = v < 0 ? -v : v;
  const double t = 1.0 - a;
  w0 = t;
  w1 = v * t * 0.5;
  w2 = -t * 0.25 + t * t * 0.5 - t * t * t / 6.0;
}

// All seven families at one offset with max |d_i| >= 2 (no box touches the
// singular point): tensor Gauss-Legendre per box, tiers glx/glw (nodes and
// weights on [0, 1] at kTierOff).  Host- and device-callable.
__host__ __device__ inline void family_far(const double d[3], const double* glx, const double* glw,
                                           double out[kNFam]) {
  double acc[kNFam] = {0, 0, 0, 0, 0, 0, 0};
  for (int box = 0; box < 8; ++box) {
    double lo[3];
    double gap2 = 0;
    for (int a = 0; a < 3; ++a) {
      lo[a] = ((box >> a) & 1) ? 0.0 : -1.0;
      const double slo = d[a] + lo[a], shi = slo + 1.0;
      const double gp = slo > 0 ? slo : (shi < 0 ? -shi : 0.0);
      gap2 += gp * gp;
    }
    const double dist = sqrt(gap2);
    int tier = kTiers - 1;
    for (int q = 0; q < kTiers; ++q)
      if (dist >= kTierDist[q]) {
        tier = q;
        break;
      }
    const int n = kTierN[tier], o = kTierOff[tier];
    // summed axis by axis (z, then y, then x) so that rounding grows with
    // the points per axis, not with their product
    double bx[kNFam] = {0, 0, 0, 0, 0, 0, 0};
    for (int i = 0; i < n; ++i) {
      const double vx = lo[0] + glx[o + i];
      double ax0, ax1, ax2;
      axis_weights(vx, ax0, ax1, ax2);
      const double X = d[0] + vx;
      double sy[5] = {0, 0, 0, 0, 0};  // over y, z: (a0 a0), (a1 a0), (a0 a1), (a2 a0), (a0 a2)
      for (int j = 0; j < n; ++j) {
        const double vy = lo[1] + glx[o + j];
        double ay0, ay1, ay2;
        axis_weights(vy, ay0, ay1, ay2);
        const double Y = d[1] + vy;
        double sz[3] = {0, 0, 0};  // over z of g times a0, a1, a2
        for (int k = 0; k < n; ++k) {
          const double vz = lo[2] + glx[o + k];
          double az0, az1, az2;
          axis_weights(vz, az0, az1, az2);
          const double Z = d[2] + vz;
          const double gw = glw[o + k] / sqrt(X * X + Y * Y + Z * Z);
          sz[0] += gw * az0;
          sz[1] += gw * az1;
          sz[2] += gw * az2;
        }
        const double wy = glw[o + j];
        sy[0] += wy * ay0 * sz[0];
        sy[1] += wy * ay1 * sz[0];
        sy[2] += wy * ay0 * sz[1];
        sy[3] += wy * ay2 * sz[0];
        sy[4] += wy * ay0 * sz[2];
      }
      const double wx = glw[o + i];
      bx[0] += wx * ax0 * sy[0];
      bx[1] += wx * ax1 * sy[0];
      bx[2] += wx * ax0 * sy[1];
      bx[3] += wx * ax0 * sy[2];
      bx[4] += wx * ax2 * sy[0];
      bx[5] += wx * ax0 * sy[3];
      bx[6] += wx * ax0 * sy[4];
    }
    for (int f = 0; f < kNFam; ++f) acc[f] += bx[f];
  }
  const double inv4pi = 0.07957747154594766788;
  for (int f = 0; f < kNFam; ++f) out[f] = acc[f] * inv4pi;
}

// out[f * Kt + idx], f < nfam, for offsets idx = (dz * Ky + dy) * Kx + dx with max |d| >= 2
__global__ void k_family_quad(int Kx, int Ky, int Kz, int nfam, double* __restrict__ out) {
  const long long Kt = (long long)Kx * Ky * Kz;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < Kt;
       idx += (long long)gridDim.x * blockDim.x) {
    const int dx = (int)(idx % Kx), dy = (int)((idx / Kx) % Ky), dz = (int)(idx / ((long long)Kx * Ky));
    if (dx < 2 && dy < 2 && dz < 2) continue;  // host computes the near offsets
    const double d[3] = {(double)dx, (double)dy, (double)dz};
    double v[kNFam];
    family_far(d, c_glx, c_glw, v);
    for (int f = 0; f < nfam; ++f) out[f * Kt + idx] = v[f];
  }
}

// ------------------------------------------------------------ near offsets --
// The 8 offsets with all d_i in {0, 1} have boxes that touch the singular
// point, so they are evaluated on the host by a reduction that needs no
// singular quadrature.  On one box (s = d + v in [a_0, a_0+1] x [a_1, a_1+1] x
// [a_2, a_2+1], integer a_i) the weight product is a polynomial in s, so the
// integral is a sum of monomial integrals J(alpha) = int_box s^alpha / |s| ds.
// s^alpha / |s| is homogeneous of degree k = |alpha| - 1, so div(s f) =
// (3 + k) f (Euler), and the divergence theorem gives
//   J(alpha) = 1 / (|alpha| + 2) * sum over faces of (s . n) int_face s^alpha / |s| dS.
// Faces through s = 0 have s . n = 0 and drop out; every other face lies at
// |s_k| >= 1 from the singular point, where the integrand is analytic, so a
// tensor Gauss-Legendre rule on the face converges geometrically (24 x 24
// points: below 1e-25 relative).  All of it runs in extended precision.

// Gauss-Legendre nodes and weights on [0, 1] in extended precision.
static void gauss_legendre01_ld(int n, long double* x, long double* w) {
  for (int i = 0; i < n; ++i) {
    long double z = cosl(3.141592653589793238462643383279502884L * (i + 0.75L) / (n + 0.5L));
    long double dp = 0;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const long double pk = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      dp = n * (z * p1 - p0) / (z * z - 1);
      const long double dz = p1 / dp;
      z -= dz;
      if (fabsl(dz) < 1e-19L) break;
    }
    x[i] = (1 - z) / 2;
    w[i] = 1 / ((1 - z * z) * dp * dp);
  }
}

// Overlap weight of one axis as a cubic in s (ascending coefficients), on
// the half of the box where sign(v) = sg, for v = s - d:
//   kind 0 (powers (0,0)): t;  kind 1 ((0,1)): v t / 2;
//   kind 2 ((1,1)): -t/4 + t^2/2 - t^3/6;  t = 1 - |v| = (1 + sg d) - sg s.
static void weight_cubic(int kind, int sg, int d, long double out[4]) {
  const long double t0 = 1.0L + sg * d, t1 = -sg;
  for (int k = 0; k < 4; ++k) out[k] = 0;
  if (kind == 0) {
    out[0] = t0;
    out[1] = t1;
  } else if (kind == 1) {  // (s - d)(t0 + t1 s) / 2
    out[0] = -d * t0 / 2;
    out[1] = (t0 - d * t1) / 2;
    out[2] = t1 / 2;
  } else {
    const long double T1[4] = {t0, t1, 0, 0};
    const long double T2[4] = {t0 * t0, 2 * t0 * t1, t1 * t1, 0};
    const long double T3[4] = {t0 * t0 * t0, 3 * t0 * t0 * t1, 3 * t0 * t1 * t1, t1 * t1 * t1};
    for (int k = 0; k < 4; ++k) out[k] = -T1[k] / 4 + T2[k] / 2 - T3[k] / 6;
  }
}

// J[(ax * 4 + ay) * 4 + az] = int over the box [a, a+1]^3 of s^alpha / |s|.
static void monomial_integrals(const int a[3], long double J[64]) {
  constexpr int n = 24;
  static long double gx[n], gw[n];
  static bool init = false;
  if (!init) {
    gauss_legendre01_ld(n, gx, gw);
    init = true;
  }
  for (int m = 0; m < 64; ++m) J[m] = 0;
  for (int k = 0; k < 3; ++k) {
    const int i = (k + 1) % 3, j = (k + 2) % 3;
    for (int side = 0; side < 2; ++side) {
      const long double c = a[k] + side;  // face s_k = c, outward normal sign: + at a+1, - at a
      const long double sn = side ? c : -c;  // s . n on this face
      if (c == 0) continue;
      // F[pk][pi][pj] = c^pk * int int s_i^pi s_j^pj / |s| over the face
      long double F[4][4] = {};
      for (int p = 0; p < n; ++p) {
        const long double si = a[i] + gx[p];
        for (int q = 0; q < n; ++q) {
          const long double sj = a[j] + gx[q];
          const long double g = gw[p] * gw[q] / sqrtl(c * c + si * si + sj * sj);
          long double pi = 1;
          for (int ei = 0; ei < 4; ++ei) {
            long double pj = 1;
            for (int ej = 0; ej < 4; ++ej) {
              F[ei][ej] += g * pi * pj;
              pj *= sj;
            }
            pi *= si;
          }
        }
      }
      long double ck = 1;
      for (int ek = 0; ek < 4; ++ek) {
        for (int ei = 0; ei < 4; ++ei)
          for (int ej = 0; ej < 4; ++ej) {
            int e[3];
            e[k] = ek;
            e[i] = ei;
            e[j] = ej;
            const int deg = ek + ei + ej;
            J[(e[0] * 4 + e[1]) * 4 + e[2]] += sn * ck * F[ei][ej] / (deg + 2);
          }
        ck *= c;
      }
    }
  }
}

// Host: all seven families at one offset with all d_i in {0, 1}.
static void family_near(const int d[3], double out[kNFam]) {
  // weight kind per family and axis: 0 (0,0), 1 (0,1), 2 (1,1)
  static const int kind[kNFam][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
                                     {2, 0, 0}, {0, 2, 0}, {0, 0, 2}};
  long double acc[kNFam] = {0, 0, 0, 0, 0, 0, 0};
  for (int box = 0; box < 8; ++box) {
    int a[3], sg[3];
    for (int ax = 0; ax < 3; ++ax) {
      const int lo = ((box >> ax) & 1) ? 0 : -1;  // v in [lo, lo + 1]
      sg[ax] = lo == 0 ? 1 : -1;
      a[ax] = d[ax] + lo;
    }
    long double J[64];
    monomial_integrals(a, J);
    for (int f = 0; f < kNFam; ++f) {
      long double wx[4], wy[4], wz[4];
      weight_cubic(kind[f][0], sg[0], d[0], wx);
      weight_cubic(kind[f][1], sg[1], d[1], wy);
      weight_cubic(kind[f][2], sg[2], d[2], wz);
      long double sum = 0;
      for (int ex = 0; ex < 4; ++ex)
        for (int ey = 0; ey < 4; ++ey)
          for (int ez = 0; ez < 4; ++ez) sum += wx[ex] * wy[ey] * wz[ez] * J[(ex * 4 + ey) * 4 + ez];
      acc[f] += sum;
    }
  }
  for (int f = 0; f < kNFam; ++f) out[f] = (double)(acc[f] / (4.0L * 3.141592653589793238462643383279502884L));
}

hipError_t family_tables(const int K[3], int nfam, double* d_out, hipStream_t s) {
  // Gauss-Legendre tiers into this device's constant memory (a few hundred bytes)
  double x[kGlTotal], w[kGlTotal];
  for (int q = 0; q < kTiers; ++q) gauss_legendre01(kTierN[q], x + kTierOff[q], w + kTierOff[q]);
  hipError_t e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_glx), x, sizeof(x), 0, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_glw), w, sizeof(w), 0, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // x, w live on this frame
  if (e != hipSuccess) return e;
  const long long Kt = (long long)K[0] * K[1] * K[2];
  hipLaunchKernelGGL(k_family_quad, dim3((unsigned)std::min<long long>((Kt + 255) / 256, 65536)), dim3(256), 0, s,
                     K[0], K[1], K[2], nfam, d_out);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // near offsets on the host
  std::vector<double> near;  // [f][8 offsets]
  std::vector<long long> idx;
  for (int dz = 0; dz < 2 && dz < K[2]; ++dz)
    for (int dy = 0; dy < 2 && dy < K[1]; ++dy)
      for (int dx = 0; dx < 2 && dx < K[0]; ++dx) {
        const int d[3] = {dx, dy, dz};
        double v[kNFam];
        family_near(d, v);
        idx.push_back(((long long)dz * K[1] + dy) * K[0] + dx);
        for (int f = 0; f < kNFam; ++f) near.push_back(v[f]);
      }
  for (size_t i = 0; i < idx.size() && e == hipSuccess; ++i)
    for (int f = 0; f < nfam && e == hipSuccess; ++f)
      e = hipMemcpyAsync(d_out + f * Kt + idx[i], &near[i * kNFam + f], sizeof(double), hipMemcpyHostToDevice, s);
  hipError_t e2 = hipStreamSynchronize(s);  // near lives on this frame
  return e != hipSuccess ? e : e2;
}

}  // namespace svh
