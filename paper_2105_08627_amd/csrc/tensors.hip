// Circulant spectrum construction and Tucker restoration kernels (gfx950).
//
//  * k_even_axis: one axis of the spectrum of the circulant embedding
//    (Sec. II.A): out[k] = sum_{n<K} w_n T[n] cos(2 pi k n / L), w_0 = 1,
//    w_n = 2 (the entries at n and L - n of the embedding); for a tensor odd
//    along the axis the same sum over n >= 1 with sin, which is the spectrum
//    divided by j.
//  * k_gemm_f64_mfma: strided batched FP64 GEMM on the matrix cores
//    (v_mfma_f64_16x16x4f64), used for the three mode products of the Tucker
//    restoration Z = core x1 F1 x2 F2 x3 F3 (eqs. 10-11).  The last product
//    writes the restored spectrum in the precision of the matvec (FP64
//    accumulation in both cases).
#include <type_traits>

#include "svh_internal.h"

namespace svh {

// out[o][k][i] for k < nk (nk = L: the whole axis; L / 2 + 1: the folded
// half, the rest following by symmetry); tab has period L.
__global__ void k_even_axis(const double* __restrict__ in, double* __restrict__ out, int nouter, int Kin,
                            int nk, int ninner, const double* __restrict__ tab, int odd, int L) {
  const size_t total = (size_t)nouter * nk * ninner;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < total;
       id += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(id % ninner);
    const size_t rest = id / ninner;
    const int k = (int)(rest % nk);
    const size_t o = rest / nk;
    const double* src = in + o * (size_t)Kin * ninner + i;
    double s = odd ? 0.0 : src[0];
    long long m = 0;
    for (int n = 1; n < Kin; ++n) {
      m += k;
      if (m >= L) m -= L;
      s += 2.0 * src[(size_t)n * ninner] * tab[m];
    }
    out[id] = s;
  }
}

__global__ void k_f64_to_f32(const double* __restrict__ in, float* __restrict__ out, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

hipError_t launch_to_f32(const double* in, float* out, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_f64_to_f32, dim3(1024), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

struct GemmArgs {
  int M, N, Kd;
  const double* A;
  long long sam, sak, sab;
  const double* B;
  long long sbk, sbn, sbb;
  void* C;
  long long scm, scn, scb;
};

typedef double double4_t __attribute__((ext_vector_type(4)));

// One wavefront per 16 x 16 output tile, row tiles fastest (the waves of one
// column strip share its B values in the caches); the operands of KS
// K-steps (KS = ceil(K / 4), at most 8) are loaded before their MFMAs.  Operand layout of
// v_mfma_f64_16x16x4f64 (wave64): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; the result register r of lane l is D[l / 16 + 4 r][l % 16]
// (checked on the device against a host product).
template <typename TOut, int KS>
__global__ void __launch_bounds__(256) k_gemm_f64_mfma(GemmArgs g) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int tiles_n = (g.N + 15) / 16, tiles_m = (g.M + 15) / 16;
  const long long tile = (long long)blockIdx.x * 4 + wave;
  if (tile >= (long long)tiles_m * tiles_n) return;
  const int tm = (int)(tile % tiles_m), tn = (int)(tile / tiles_m);
  const long long b = blockIdx.y;
  const double* A = g.A + b * g.sab;
  const double* Bm = g.B + b * g.sbb;
  TOut* C = static_cast<TOut*>(g.C) + b * g.scb;
  const int col = tn * 16 + (lane & 15), row = tm * 16 + (lane & 15);
  const int kq = lane >> 4;
  // clamped addresses (always valid), zeros selected after the loads
  const int rowc = row < g.M ? row : g.M - 1, colc = col < g.N ? col : g.N - 1;
  double4_t acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < g.Kd; k0 += 4 * KS) {
    double a[KS], bv[KS];
#pragma unroll
    for (int st = 0; st < KS; ++st) {
      const int kk = k0 + 4 * st + kq;
      const int kc = kk < g.Kd ? kk : g.Kd - 1;
      a[st] = A[rowc * g.sam + kc * g.sak];
      bv[st] = Bm[kc * g.sbk + colc * g.sbn];
    }
#pragma unroll
    for (int st = 0; st < KS; ++st) {
      const int kk = k0 + 4 * st + kq;
      const bool ok = kk < g.Kd;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64((ok && row < g.M) ? a[st] : 0.0, (ok && col < g.N) ? bv[st] : 0.0,
                                                 acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int orow = tm * 16 + kq + 4 * r;
    if (orow < g.M && col < g.N) C[orow * g.scm + col * g.scn] = (TOut)acc[r];
  }
}

static hipError_t gemm(const GemmArgs& g, int batch, bool f32out, hipStream_t s) {
  const long long tiles = (long long)((g.M + 15) / 16) * ((g.N + 15) / 16);
  dim3 grid((unsigned)((tiles + 3) / 4), batch);
  const int steps = (g.Kd + 3) / 4;
  auto go = [&](auto kst) {
    constexpr int KS = decltype(kst)::value;
    if (f32out) hipLaunchKernelGGL((k_gemm_f64_mfma<float, KS>), grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL((k_gemm_f64_mfma<double, KS>), grid, dim3(256), 0, s, g);
  };
  switch (steps < 8 ? steps : 8) {
    case 1: go(std::integral_constant<int, 1>{}); break;
    case 2: go(std::integral_constant<int, 2>{}); break;
    case 3: go(std::integral_constant<int, 3>{}); break;
    case 4: go(std::integral_constant<int, 4>{}); break;
    case 5: go(std::integral_constant<int, 5>{}); break;
    case 6: go(std::integral_constant<int, 6>{}); break;
    case 7: go(std::integral_constant<int, 7>{}); break;
    default: go(std::integral_constant<int, 8>{}); break;
  }
  return hipGetLastError();
}

hipError_t launch_even_spectrum(const svh_problem* p, const double* d_T, double* d_out, double* d_tmp1,
                                double* d_tmp2, hipStream_t s) {
  // cos tables are built per call (setup only)
  const int Kx = p->K[0], Ky = p->K[1], Kz = p->K[2];
  const int Lx = p->L[0], Ly = p->L[1], Lz = p->L[2];
  std::vector<double> tab;
  double* d_cos = nullptr;
  const int Lmax = std::max(Lx, std::max(Ly, Lz));
  hipError_t e = hipMalloc(&d_cos, sizeof(double) * 3 * Lmax);
  if (e != hipSuccess) return e;
  tab.assign(3 * (size_t)Lmax, 0.0);
  for (int a = 0; a < 3; ++a)
    for (int m = 0; m < p->L[a]; ++m)
      tab[(size_t)a * Lmax + m] = (double)cosl(2.0L * 3.141592653589793238462643383279502884L * m / p->L[a]);
  e = hipMemcpyAsync(d_cos, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    // x: [Kz][Ky][Kx] -> [Kz][Ky][Lx]
    hipLaunchKernelGGL(k_even_axis, dim3(2048), dim3(256), 0, s, d_T, d_tmp1, Kz * Ky, Kx, Lx, 1, d_cos, 0, Lx);
    // y: [Kz][Ky][Lx] -> [Kz][Ly][Lx]  (this is the z-space kernel)
    hipLaunchKernelGGL(k_even_axis, dim3(2048), dim3(256), 0, s, d_tmp1, d_tmp2, Kz, Ky, Ly, Lx,
                       d_cos + Lmax, 0, Ly);
    // z: [Kz][Ly][Lx] -> [Lz][Ly][Lx]
    if (d_out)
      hipLaunchKernelGGL(k_even_axis, dim3(2048), dim3(256), 0, s, d_tmp2, d_out, 1, Kz, Lz, Ly * Lx,
                         d_cos + 2 * Lmax, 0, Lz);
    e = hipGetLastError();
  }
  hipError_t e2 = hipStreamSynchronize(s);
  hipFree(d_cos);
  return e != hipSuccess ? e : e2;
}

// Folded spectra of nfam family tables d_in [f][Kz][Ky][Kx] (M0, M1x, M1y,
// M1z, M2x, M2y, M2z in that order): d_out[f][kz][ky][kx] for k_a <= L_a / 2,
// each axis a cosine sum (or, along the odd axis of an M1 family, the sine
// sum: the spectrum divided by j).  d_tmp: Kz*Ky*(Lx/2+1) + Kz*(Ly/2+1)*(Lx/2+1)
// doubles.  Synchronises the stream.
hipError_t launch_folded_spectra(const svh_problem* p, const double* d_in, int nfam, double* d_out, double* d_tmp,
                                 hipStream_t s) {
  const int Kx = p->K[0], Ky = p->K[1], Kz = p->K[2];
  const int Lx = p->L[0], Ly = p->L[1], Lz = p->L[2];
  const int hx = Lx / 2 + 1, hy = Ly / 2 + 1, hz = Lz / 2 + 1;
  const int Lmax = std::max(Lx, std::max(Ly, Lz));
  std::vector<double> tab(6 * (size_t)Lmax, 0.0);  // cos, sin per axis
  for (int a = 0; a < 3; ++a)
    for (int m = 0; m < p->L[a]; ++m) {
      const long double ang = 2.0L * 3.141592653589793238462643383279502884L * m / p->L[a];
      tab[(size_t)(2 * a) * Lmax + m] = (double)cosl(ang);
      tab[(size_t)(2 * a + 1) * Lmax + m] = (double)sinl(ang);
    }
  double* d_tab = nullptr;
  hipError_t e = hipMalloc(&d_tab, sizeof(double) * tab.size());
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(d_tab, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice, s);
  double* t1 = d_tmp;
  double* t2 = d_tmp + (size_t)Kz * Ky * hx;
  const size_t Kt = (size_t)Kx * Ky * Kz, Ht = (size_t)hx * hy * hz;
  for (int f = 0; f < nfam && e == hipSuccess; ++f) {
    const int ox = f == 1, oy = f == 2, oz = f == 3;
    hipLaunchKernelGGL(k_even_axis, dim3(2048), dim3(256), 0, s, d_in + f * Kt, t1, Kz * Ky, Kx, hx, 1,
                       d_tab + (size_t)ox * Lmax, ox, Lx);
    hipLaunchKernelGGL(k_even_axis, dim3(2048), dim3(256), 0, s, t1, t2, Kz, Ky, hy, hx,
                       d_tab + (size_t)(2 + oy) * Lmax, oy, Ly);
    hipLaunchKernelGGL(k_even_axis, dim3(2048), dim3(256), 0, s, t2, d_out + f * Ht, 1, Kz, hz, hy * hx,
                       d_tab + (size_t)(4 + oz) * Lmax, oz, Lz);
    e = hipGetLastError();
  }
  hipError_t e2 = hipStreamSynchronize(s);
  hipFree(d_tab);
  return e != hipSuccess ? e : e2;
}

size_t folded_size(const svh_problem* p) {
  return (size_t)(p->L[0] / 2 + 1) * (p->L[1] / 2 + 1) * (p->L[2] / 2 + 1);
}

size_t tucker_scratch_doubles(const svh_problem* p) {
  const DevTucker& t = p->tk;
  return (size_t)p->L[0] * t.d[1] * t.d[2] + (size_t)p->L[0] * p->L[1] * t.d[2];
}

size_t tucker_scratch_doubles5(const svh_problem* p) {
  size_t m = 0;
  for (int f = 0; f < kNFam; ++f) {
    const DevTucker& t = p->tk5[f];
    m = std::max(m, (size_t)p->L[0] * t.d[1] * t.d[2] + (size_t)p->L[0] * p->L[1] * t.d[2]);
  }
  return m;
}

hipError_t launch_tucker_box(int n1, int n2, int n3, const DevTucker& t, const double* F3, bool fp32_out,
                             void* d_out, double* d_V, double* d_W, hipStream_t s) {
  // out[k3][k2][k1] = sum core[c][b][a] F1[k1][a] F2[k2][b] F3[k3][c], k_i < n_i
  const int d1 = t.d[0], d2 = t.d[1], d3 = t.d[2];
  hipError_t e;
  GemmArgs g1{n1, d2 * d3, d1, t.F[0], d1, 1, 0, t.core, 1, d1, 0, d_V, (long long)d2 * d3, 1, 0};
  if ((e = gemm(g1, 1, false, s)) != hipSuccess) return e;
  GemmArgs g2{n2, d3, d2, t.F[1], d2, 1, 0, d_V, 1, d2, (long long)d2 * d3, d_W, (long long)n1 * d3, 1, d3};
  if ((e = gemm(g2, n1, false, s)) != hipSuccess) return e;
  GemmArgs g3{n3, n1 * n2, d3, F3, d3, 1, 0, d_W, 1, d3, 0, d_out, (long long)n1 * n2, 1, 0};
  return gemm(g3, 1, fp32_out, s);
}

hipError_t launch_tucker_rebuild_rows(const svh_problem* p, const DevTucker& t, const double* Fz3, int M3,
                                      bool fp32_out, void* d_out, double* d_V, double* d_W, hipStream_t s,
                                      bool xy_transposed) {
  const int L1 = p->L[0], L2 = p->L[1];
  const int d1 = t.d[0], d2 = t.d[1], d3 = t.d[2];
  hipError_t e;
  GemmArgs g1{L1, d2 * d3, d1, t.F[0], d1, 1, 0, t.core, 1, d1, 0, d_V, (long long)d2 * d3, 1, 0};
  if ((e = gemm(g1, 1, false, s)) != hipSuccess) return e;
  // W[ky][kx][c] (or W[kx][ky][c] when transposed) = sum_b F2[ky][b] V[kx][c][b]
  const long long scm = xy_transposed ? d3 : (long long)L1 * d3;
  const long long scb = xy_transposed ? (long long)L2 * d3 : d3;
  GemmArgs g2{L2, d3, d2, t.F[1], d2, 1, 0, d_V, 1, d2, (long long)d2 * d3, d_W, scm, 1, scb};
  if ((e = gemm(g2, L1, false, s)) != hipSuccess) return e;
  GemmArgs g3{M3, L1 * L2, d3, Fz3, d3, 1, 0, d_W, 1, d3, 0, d_out, (long long)L1 * L2, 1, 0};
  return gemm(g3, 1, fp32_out, s);
}

hipError_t launch_tucker_rebuild(const svh_problem* p, bool fp32_out, bool zspace, void* d_out, double* d_V,
                                 double* d_W, hipStream_t s) {
  // Z[kz][ky][kx] = sum_c F3[kz][c] W[ky][kx][c]; in z space the third
  // factor is its inverse z transform and only offsets dz < Kz are restored
  const DevTucker& t = p->tk;
  return launch_tucker_rebuild_rows(p, t, zspace ? t.Fz : t.F[2], zspace ? p->K[2] : p->L[2], fp32_out, d_out,
                                    d_V, d_W, s);
}

__global__ void k_gather_t(const double* __restrict__ in, double* __restrict__ out, const int32_t* __restrict__ dz,
                           int nd, int Lx, int Ly) {
  const size_t total = (size_t)nd * Lx * Ly;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < total; id += (size_t)gridDim.x * blockDim.x) {
    const int ky = (int)(id % Ly);
    const size_t rest = id / Ly;
    const int kx = (int)(rest % Lx);
    const int q = (int)(rest / Lx);
    out[id] = in[((size_t)dz[q] * Ly + ky) * Lx + kx];
  }
}

hipError_t launch_gather_transposed(const svh_problem* p, const double* d_in, double* d_out, hipStream_t s) {
  int32_t* d_dz = nullptr;
  const int nd = (int)p->dzset.size();
  hipError_t e = hipMalloc(&d_dz, sizeof(int32_t) * nd);
  if (e != hipSuccess) return e;
  e = hipMemcpy(d_dz, p->dzset.data(), sizeof(int32_t) * nd, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_gather_t, dim3(2048), dim3(256), 0, s, d_in, d_out, d_dz, nd, p->L[0], p->L[1]);
    e = hipGetLastError();
  }
  hipError_t e2 = hipStreamSynchronize(s);
  hipFree(d_dz);
  return e != hipSuccess ? e : e2;
}

// Parity of the seven families per axis (x, y, z): M1 of axis a is odd along a.
static const int kFamOdd[kNFam][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
                                      {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};

hipError_t launch_zspace_families(const svh_problem* p, const double* d_rows, int nd, double* d_out,
                                  double* d_tmp, hipStream_t s) {
  const int Kx = p->K[0], Ky = p->K[1];
  const int Lx = p->L[0], Ly = p->L[1];
  const int Lmax = std::max(Lx, Ly);
  std::vector<double> tab(4 * (size_t)Lmax, 0.0);  // cos x, sin x, cos y, sin y
  for (int a = 0; a < 2; ++a)
    for (int m = 0; m < p->L[a]; ++m) {
      const long double ang = 2.0L * 3.141592653589793238462643383279502884L * m / p->L[a];
      tab[(size_t)(2 * a) * Lmax + m] = (double)cosl(ang);
      tab[(size_t)(2 * a + 1) * Lmax + m] = (double)sinl(ang);
    }
  double* d_tab = nullptr;
  hipError_t e = hipMalloc(&d_tab, sizeof(double) * tab.size());
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(d_tab, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice, s);
  for (int f = 0; f < kNFam && e == hipSuccess; ++f) {
    const double* in = d_rows + (size_t)f * nd * Ky * Kx;
    double* out = d_out + (size_t)f * nd * Ly * Lx;
    const int ox = kFamOdd[f][0], oy = kFamOdd[f][1];
    // x: [nd][Ky][Kx] -> [nd][Ky][Lx]
    hipLaunchKernelGGL(k_even_axis, dim3(2048), dim3(256), 0, s, in, d_tmp, nd * Ky, Kx, Lx, 1,
                       d_tab + (size_t)ox * Lmax, ox, Lx);
    // y: [nd][Ky][Lx] -> [nd][Ly][Lx]
    hipLaunchKernelGGL(k_even_axis, dim3(2048), dim3(256), 0, s, d_tmp, out, nd, Ky, Ly, Lx,
                       d_tab + (size_t)(2 + oy) * Lmax, oy, Ly);
    e = hipGetLastError();
  }
  hipError_t e2 = hipStreamSynchronize(s);
  hipFree(d_tab);
  return e != hipSuccess ? e : e2;
}

}  // namespace svh
