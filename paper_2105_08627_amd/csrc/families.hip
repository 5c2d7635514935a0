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
// with all d_i in {0, 1} are computed on the host: boxes with the singular
// point at a corner use the Duffy pyramid map, which removes the 1/r
// singularity.
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

// Host: all seven families at one offset with all d_i in {0, 1}.
static void family_near(const int d[3], double out[kNFam]) {
  static std::vector<double> xa, wa, xr, wr, xg, wg;
  if (xa.empty()) {
    xa.resize(24); wa.resize(24); xr.resize(16); wr.resize(16); xg.resize(20); wg.resize(20);
    gauss_legendre01(24, xa.data(), wa.data());
    gauss_legendre01(16, xr.data(), wr.data());
    gauss_legendre01(20, xg.data(), wg.data());
  }
  long double acc[kNFam] = {0, 0, 0, 0, 0, 0, 0};  // extended precision: ~2e5 terms per family
  auto add = [&](double vx, double vy, double vz, double wt) {
    double ax[3], ay[3], az[3];
    axis_weights(vx, ax[0], ax[1], ax[2]);
    axis_weights(vy, ay[0], ay[1], ay[2]);
    axis_weights(vz, az[0], az[1], az[2]);
    acc[0] += wt * ax[0] * ay[0] * az[0];
    acc[1] += wt * ax[1] * ay[0] * az[0];
    acc[2] += wt * ax[0] * ay[1] * az[0];
    acc[3] += wt * ax[0] * ay[0] * az[1];
    acc[4] += wt * ax[2] * ay[0] * az[0];
    acc[5] += wt * ax[0] * ay[2] * az[0];
    acc[6] += wt * ax[0] * ay[0] * az[2];
  };
  for (int box = 0; box < 8; ++box) {
    double lo[3], slo[3];
    bool corner = true;
    for (int a = 0; a < 3; ++a) {
      lo[a] = ((box >> a) & 1) ? 0.0 : -1.0;
      slo[a] = d[a] + lo[a];
      if (!(slo[a] == 0.0 || slo[a] == -1.0)) corner = false;  // 0 must be an endpoint
    }
    if (corner) {
      // s-box is [0,1] or [-1,0] per axis; s = sign * t, t in [0,1]^3;
      // pyramid `ax`: t = rho (.., 1 at ax, ..) scaled by (e1, e2) on the others
      double sg[3];
      for (int a = 0; a < 3; ++a) sg[a] = slo[a] == 0.0 ? 1.0 : -1.0;
      for (int ax = 0; ax < 3; ++ax) {
        const int o1 = (ax + 1) % 3, o2 = (ax + 2) % 3;
        for (int ir = 0; ir < 16; ++ir)
          for (int i1 = 0; i1 < 24; ++i1)
            for (int i2 = 0; i2 < 24; ++i2) {
              const double rho = xr[ir], e1 = xa[i1], e2 = xa[i2];
              double t[3];
              t[ax] = rho;
              t[o1] = rho * e1;
              t[o2] = rho * e2;
              const double wt = wr[ir] * wa[i1] * wa[i2] * rho / std::sqrt(1.0 + e1 * e1 + e2 * e2);
              add(sg[0] * t[0] - d[0], sg[1] * t[1] - d[1], sg[2] * t[2] - d[2], wt);
            }
      }
    } else {
      for (int i = 0; i < 20; ++i)
        for (int j = 0; j < 20; ++j)
          for (int k = 0; k < 20; ++k) {
            const double vx = lo[0] + xg[i], vy = lo[1] + xg[j], vz = lo[2] + xg[k];
            const double X = d[0] + vx, Y = d[1] + vy, Z = d[2] + vz;
            add(vx, vy, vz, wg[i] * wg[j] * wg[k] / std::sqrt(X * X + Y * Y + Z * Z));
          }
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
