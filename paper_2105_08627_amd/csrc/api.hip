// C ABI entry points (include/svh.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>

#include "host_math.h"
#include "svh_internal.h"

namespace svh {
bool make_plan(int L, FftPlan& p) {
  p = FftPlan();
  p.L = L;
  int n = L;
  const int rad[4] = {8, 4, 2, 3};
  for (int q = 0; q < 4; ++q) {
    const int r = rad[q];
    while (n % r == 0) {
      if (r == 2 && n % 4 == 0) break;
      if (p.ns >= kMaxStages) return false;
      p.r[p.ns++] = r;
      n /= r;
    }
  }
  if (n != 1 || p.ns == 0) return false;
  p.tp = L;
  for (int s = 0; s < p.ns; ++s) p.tp = std::min(p.tp, L / p.r[s]);
  return true;
}

FftPlan reversed(const FftPlan& p) {
  FftPlan q = p;
  for (int s = 0; s < p.ns; ++s) q.r[s] = p.r[p.ns - 1 - s];
  return q;
}

bool supported_length(int L) {
  if (L < 2 || L > 1024) return false;
  int n = L;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}
}  // namespace svh

using namespace svh;

namespace {

svh_status fail(svh_problem* p, svh_status st, const std::string& msg) {
  if (p) p->err = msg;
  return st;
}

#define HIPCHK(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(p, e_ == hipErrorOutOfMemory ? SVH_ENOMEM : SVH_EHIP,                    \
                  std::string(#call) + ": " + hipGetErrorString(e_));                      \
  } while (0)

template <typename T>
hipError_t upload(T** dst, const T* src, size_t n) {
  if (*dst) {
    hipFree(*dst);
    *dst = nullptr;
  }
  if (n == 0) return hipSuccess;
  hipError_t e = hipMalloc(dst, n * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
}

template <typename T>
void dfree(T*& ptr) {
  if (ptr) hipFree(ptr);
  ptr = nullptr;
}

// FFT length of an axis with K voxels: at least 2K - 1 (a linear convolution),
// so an even length is at least 2K.  The x passes rely on this: with an even
// radix the upper half of the first forward butterflies and of the last
// inverse butterflies lies in the zero padding (positions >= L/2 >= K).
int choose_length(int K) {
  if (supported_length(2 * K)) return 2 * K;
  for (int L = std::max(2, 2 * K - 1);; ++L)
    if (supported_length(L)) return L;
}

void free_dev_tucker(DevTucker& t) {
  dfree(t.core);
  dfree(t.Fz);
  dfree(t.Fzd);
  for (int a = 0; a < 3; ++a) dfree(t.F[a]);
  t = DevTucker();
}

void free_tucker(svh_problem* p) {
  free_dev_tucker(p->tk);
  for (int f = 0; f < kNFam; ++f) free_dev_tucker(p->tk5[f]);
  p->tucker = false;
}

// Parity of the seven families per axis (x, y, z): M1 of axis a is odd along a.
const int kOdd[kNFam][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};

// Inverse z transform of the third Tucker factor at the plane offsets dz:
// Fz[m][c] = (1/Lz) sum_kz F3[kz][c] cos(2 pi kz dz_m / Lz) for an even
// family, the same with sin for a family odd in z (whose spectrum is j F).
std::vector<double> zspace_factor(const TuckerFactors& tf, int Lz, const std::vector<int>& dz, bool odd) {
  const int d3 = tf.d[2];
  std::vector<double> Fz(dz.size() * (size_t)d3);
  for (size_t m = 0; m < dz.size(); ++m)
    for (int c = 0; c < d3; ++c) {
      long double acc = 0;
      for (int kz = 0; kz < Lz; ++kz) {
        const long long r = ((long long)kz * dz[m]) % Lz;
        const long double a = 2.0L * 3.141592653589793238462643383279502884L * r / Lz;
        acc += (long double)tf.F[2][(size_t)kz * d3 + c] * (odd ? sinl(a) : cosl(a));
      }
      Fz[m * d3 + c] = (double)(acc / Lz);
    }
  return Fz;
}

size_t vec_bytes_AB(const svh_problem* p, size_t csize) {
  const size_t nzp = p->zlist.size();
  const Geo g = make_geo(p, csize);
  return nzp * (size_t)(g.pa + g.pb) * csize;
}

int chunk_rhs(const svh_problem* p, int nrhs) {
  int maxr = kMaxVecsPerChunk / p->C;
  if (p->C == 5 && maxr > 8) maxr -= maxr % 8;  // the five-component z step takes right-hand sides 8 at a time
  return std::max(1, std::min(nrhs, maxr));
}

// Workspace of svh_matvec_noalloc: a fixed array in device memory, one copy
// per device the library runs on, held until the process ends.  Host code
// never passes `scratch` itself to a kernel (on the host the name is only a
// stand-in for the symbol): it looks up each device's address once, with
// that device current, and uses that address.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

// Address of `scratch` on device dev, which must be the current device.
hipError_t scratch_address(int dev, void** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

svh_status svh_create(svh_problem** out, int Kx, int Ky, int Kz, double dx_m, int basis,
                      const uint8_t* mask_host) {
  if (!out) return SVH_EINVAL;
  *out = nullptr;
  if (Kx < 1 || Ky < 1 || Kz < 1 || !(dx_m > 0) || !mask_host) return SVH_EINVAL;
  if (basis != 3 && basis != 5) return SVH_EINVAL;
  if (Kx > 512 || Ky > 512 || Kz > 512) return SVH_EINVAL;
  std::unique_ptr<svh_problem> up(new svh_problem());
  svh_problem* p = up.get();
  p->K[0] = Kx;
  p->K[1] = Ky;
  p->K[2] = Kz;
  p->dx = dx_m;
  p->basis = basis;
  p->C = basis;
  HIPCHK(hipGetDevice(&p->device));
  HIPCHK(hipDeviceGetAttribute(&p->ncu, hipDeviceAttributeMultiprocessorCount, p->device));
  HIPCHK(hipDeviceGetAttribute(&p->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device));
  {
    void* sp = nullptr;  // set-up of this device's svh_matvec_noalloc workspace
    HIPCHK(scratch_address(p->device, &sp));
  }
  const size_t Kt = (size_t)Kx * Ky * Kz;
  p->vidx.assign(Kt, -1);
  int n = 0;
  std::vector<char> zocc(Kz, 0);
  for (int z = 0; z < Kz; ++z)
    for (int y = 0; y < Ky; ++y)
      for (int x = 0; x < Kx; ++x) {
        const size_t i = ((size_t)z * Ky + y) * Kx + x;
        if (mask_host[i]) {
          p->vidx[i] = n++;
          zocc[z] = 1;
        }
      }
  if (n == 0) return SVH_EINVAL;
  p->nvox = n;
  for (int a = 0; a < 3; ++a) {
    p->L[a] = choose_length(p->K[a]);
    if (!make_plan(p->L[a], p->plan[a])) return SVH_EINVAL;
  }
  for (int z = 0; z < Kz; ++z)
    if (zocc[z]) p->zlist.push_back(z);
  p->zslot.assign(p->L[2], -1);
  for (size_t s = 0; s < p->zlist.size(); ++s) p->zslot[p->zlist[s]] = (int32_t)s;
  if (p->zlist.size() <= (size_t)kMaxDirectPlanes) {
    // distinct plane offsets |z_i - z_j| and the per-(i, j) slot codes of the
    // coupled z step
    const int nzp = (int)p->zlist.size();
    std::vector<int> slot(Kz, -1);
    for (int i = 0; i < nzp; ++i)
      for (int j = 0; j < nzp; ++j) slot[std::abs(p->zlist[i] - p->zlist[j])] = 1;
    for (int d = 0; d < Kz; ++d)
      if (slot[d] >= 0) {
        slot[d] = (int)p->dzset.size();
        p->dzset.push_back(d);
      }
    if (p->dzset.size() <= (size_t)kMaxDz5) {
      std::vector<uint8_t> q(32 * 32, 0);
      for (int i = 0; i < nzp; ++i)
        for (int j = 0; j < nzp; ++j) {
          const int d = p->zlist[j] - p->zlist[i];
          q[i * 32 + j] = (uint8_t)(slot[std::abs(d)] | (d < 0 ? 0x80 : 0));
        }
      HIPCHK(upload(&p->d_qtab, q.data(), q.size()));
    }
  }
  if (basis == 3 && p->d_qtab) {
    // frequency phases of the fused y / z / inverse-y step per precision and
    // the twiddles of the phase length Ly / phases
    p->fused_r[SVH_FP64] = fused_phases(p, sizeof(double2), sizeof(double));
    p->fused_r[SVH_FP32] = fused_phases(p, sizeof(float2), sizeof(float));
    p->fused2_r = yzy2_phases(p);
    if (p->fused_r[0] > 0 && p->fused_r[1] > 0) {
      const int P64 = p->L[1] / p->fused_r[0], P32 = p->L[1] / p->fused_r[1];
      std::vector<double2> t64(P64);
      std::vector<float2> t32(P32);
      for (int m = 0; m < P64; ++m) {
        const long double ang = 2.0L * 3.141592653589793238462643383279502884L * m / P64;
        t64[m] = make_double2((double)cosl(ang), (double)-sinl(ang));
      }
      for (int m = 0; m < P32; ++m) {
        const long double ang = 2.0L * 3.141592653589793238462643383279502884L * m / P32;
        t32[m] = make_float2((float)cosl(ang), (float)-sinl(ang));
      }
      HIPCHK(upload(&p->d_twp64, t64.data(), t64.size()));
      HIPCHK(upload(&p->d_twp32, t32.data(), t32.size()));
    }
  }
  {
    // occupancy words of the rows of the occupied planes (x pass gather and
    // inverse x pass scatter)
    const int nw = (Kx + 63) / 64, nzp = (int)p->zlist.size();
    p->xrow_words = nw;
    // one extra all-zero word at the end: the zero value that the x pass
    // loads for empty grid positions
    std::vector<XRowWord> xr((size_t)nzp * Ky * nw + 1, XRowWord{0, 0, 0});
    for (int zp = 0; zp < nzp; ++zp)
      for (int y = 0; y < Ky; ++y)
        for (int w = 0; w < nw; ++w) {
          XRowWord& e = xr[((size_t)zp * Ky + y) * nw + w];
          e.bits = 0;
          e.base = 0;
          e.pad = 0;
          bool first = true;
          for (int b = 0; b < 64 && w * 64 + b < Kx; ++b) {
            const int32_t k = p->vidx[((size_t)p->zlist[zp] * Ky + y) * Kx + w * 64 + b];
            if (k < 0) continue;
            if (first) e.base = k;
            first = false;
            e.bits |= 1ull << b;
          }
        }
    HIPCHK(upload(&p->d_xrow, xr.data(), xr.size()));
  }
  HIPCHK(upload(&p->d_zlist, p->zlist.data(), p->zlist.size()));
  HIPCHK(upload(&p->d_zslot, p->zslot.data(), p->zslot.size()));
  for (int a = 0; a < 3; ++a) {
    const int L = p->L[a];
    std::vector<double2> t64(L);
    std::vector<float2> t32(L);
    for (int m = 0; m < L; ++m) {
      const long double ang = 2.0L * 3.141592653589793238462643383279502884L * m / L;
      t64[m] = make_double2((double)cosl(ang), (double)-sinl(ang));
      t32[m] = make_float2((float)cosl(ang), (float)-sinl(ang));
    }
    HIPCHK(upload(&p->d_tw64[a], t64.data(), L));
    HIPCHK(upload(&p->d_tw32[a], t32.data(), L));
  }
  *out = up.release();
  return SVH_OK;
}

svh_status svh_get_sizes(const svh_problem* p, int* K, int* Lx, int* Ly, int* Lz) {
  if (!p) return SVH_EINVAL;
  if (K) *K = p->nvox;
  if (Lx) *Lx = p->L[0];
  if (Ly) *Ly = p->L[1];
  if (Lz) *Lz = p->L[2];
  return SVH_OK;
}

svh_status svh_set_material(svh_problem* p, int nfreq, const double* f_hz, const double* sigma0,
                            const double* lambda, int per_voxel) {
  if (!p) return SVH_EINVAL;
  if (nfreq < 1 || !f_hz || !sigma0 || !lambda) return fail(p, SVH_EINVAL, "set_material: bad arguments");
  const int K = p->nvox;
  // validate everything before any state of p changes
  for (int f = 0; f < nfreq; ++f)
    if (!(f_hz[f] > 0) || !std::isfinite(f_hz[f])) return fail(p, SVH_EINVAL, "set_material: frequency must be > 0");
  for (int k = 0; k < (per_voxel ? K : 1); ++k)
    if (!(sigma0[k] >= 0) || !(lambda[k] > 0) || !std::isfinite(sigma0[k]) || !std::isfinite(lambda[k]))
      return fail(p, SVH_EINVAL, "set_material: need sigma0 >= 0, lambda > 0");
  std::vector<double2> cd64((size_t)nfreq * K);
  std::vector<float2> cd32((size_t)nfreq * K);
  std::vector<double2> s64(nfreq);
  std::vector<float2> s32(nfreq);
  std::vector<std::complex<double>> sconv(nfreq);
  for (int f = 0; f < nfreq; ++f) {
    const double w = 2 * M_PI * f_hz[f];
    const std::complex<double> s(0.0, w * kMu0 * p->dx);
    sconv[f] = s;
    s64[f] = make_double2(s.real(), s.imag());
    s32[f] = make_float2((float)s.real(), (float)s.imag());
    for (int k = 0; k < K; ++k) {
      const double s0 = sigma0[per_voxel ? k : 0];
      const double lam = lambda[per_voxel ? k : 0];
      // eq. 3: sigma = sigma0 - j / (w mu lam^2); c = 1 / sigma
      const std::complex<double> sigma(s0, -1.0 / (w * kMu0 * lam * lam));
      const std::complex<double> c = 1.0 / sigma / p->dx;
      cd64[(size_t)f * K + k] = make_double2(c.real(), c.imag());
      cd32[(size_t)f * K + k] = make_float2((float)c.real(), (float)c.imag());
    }
  }
  // a failed upload leaves the material unset rather than half replaced
  p->nfreq = 0;
  p->sconv.clear();
  p->cdiag_host.clear();
  p->diag_freq = -2;
  HIPCHK(upload(&p->d_cdiag64, cd64.data(), cd64.size()));
  HIPCHK(upload(&p->d_cdiag32, cd32.data(), cd32.size()));
  HIPCHK(upload(&p->d_sconv64, s64.data(), s64.size()));
  HIPCHK(upload(&p->d_sconv32, s32.data(), s32.size()));
  p->sconv = std::move(sconv);
  p->cdiag_host.resize(cd64.size());
  for (size_t i = 0; i < cd64.size(); ++i) p->cdiag_host[i] = std::complex<double>(cd64[i].x, cd64[i].y);
  p->nfreq = nfreq;
  p->diag_freq = -2;
  return SVH_OK;
}

namespace {
// Piecewise-linear basis: the seven family tables and their z-space kernels at
// the occupied plane offsets.
svh_status setup_tensors5(svh_problem* p, hipStream_t s) {
  const int nzp = (int)p->zlist.size();
  const bool direct = nzp <= kMaxDirectPlanes && p->d_qtab;  // the direct z step applies
  const size_t Kt = (size_t)p->K[0] * p->K[1] * p->K[2];
  const int nd = direct ? (int)p->dzset.size() : 0;
  const size_t rows = (size_t)nd * p->K[1] * p->K[0];
  const size_t gsz = (size_t)kNFam * nd * p->L[1] * p->L[0];
  const size_t hsz = folded_size(p);
  double *dF = nullptr, *dR = nullptr, *dT = nullptr;
  HIPCHK(hipMalloc(&dF, kNFam * Kt * sizeof(double)));
  hipError_t e = p->store.empty() ? family_tables(p->K, kNFam, dF, s) : store_tables(p, kNFam, dF, s);
  p->Tf.assign(kNFam * Kt, 0.0);
  if (e == hipSuccess) e = hipMemcpy(p->Tf.data(), dF, kNFam * Kt * sizeof(double), hipMemcpyDeviceToHost);
  // folded spectra of the seven families (z FFT step)
  if (e == hipSuccess) e = hipMalloc(&p->d_zhat64, kNFam * hsz * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&p->d_zhat32, kNFam * hsz * sizeof(float));
  if (e == hipSuccess) {
    const size_t nt = (size_t)p->K[2] * (p->L[0] / 2 + 1) * (p->K[1] + p->L[1] / 2 + 1);
    e = hipMalloc(&dT, nt * sizeof(double));
  }
  if (e == hipSuccess) e = launch_folded_spectra(p, dF, kNFam, p->d_zhat64, dT, s);
  if (e == hipSuccess) e = launch_to_f32(p->d_zhat64, p->d_zhat32, kNFam * hsz, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipFree(dF);
  if (dT) hipFree(dT);
  dT = nullptr;
  HIPCHK(e);
  // M0 from the closed form if chosen, else from the same quadrature; exact
  // zeros where an odd family vanishes
  if (p->green == SVH_GREEN_CLOSED_FORM && p->store.empty()) std::copy(p->T.begin(), p->T.end(), p->Tf.begin());
  else std::copy(p->Tf.begin(), p->Tf.begin() + Kt, p->T.begin());
  for (int f = 1; f <= 3; ++f) {
    const int a = f - 1;
    for (int z = 0; z < p->K[2]; ++z)
      for (int y = 0; y < p->K[1]; ++y)
        for (int x = 0; x < p->K[0]; ++x) {
          const int d[3] = {x, y, z};
          if (d[a] == 0) p->Tf[f * Kt + ((size_t)z * p->K[1] + y) * p->K[0] + x] = 0.0;
        }
  }
  if (!direct) return SVH_OK;
  std::vector<double> hr(kNFam * rows);
  for (int f = 0; f < kNFam; ++f)
    for (int q = 0; q < nd; ++q)
      std::copy(p->Tf.begin() + f * Kt + (size_t)p->dzset[q] * p->K[1] * p->K[0],
                p->Tf.begin() + f * Kt + (size_t)(p->dzset[q] + 1) * p->K[1] * p->K[0],
                hr.begin() + ((size_t)f * nd + q) * p->K[1] * p->K[0]);
  HIPCHK(hipMalloc(&p->d_g5_64, gsz * sizeof(double)));
  HIPCHK(hipMalloc(&p->d_g5_32, gsz * sizeof(float)));
  HIPCHK(hipMalloc(&dR, hr.size() * sizeof(double)));
  e = hipMalloc(&dT, (size_t)nd * p->K[1] * p->L[0] * sizeof(double));
  if (e == hipSuccess) e = hipMemcpy(dR, hr.data(), hr.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_zspace_families(p, dR, nd, p->d_g5_64, dT, s);
  if (e == hipSuccess) e = launch_to_f32(p->d_g5_64, p->d_g5_32, gsz, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipFree(dR);
  if (dT) hipFree(dT);
  HIPCHK(e);
  return SVH_OK;
}
}  // namespace

svh_status svh_setup_tensors(svh_problem* p, void* stream) {
  if (!p) return SVH_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t Kt = (size_t)p->K[0] * p->K[1] * p->K[2];
  p->T.assign(Kt, 0.0);
  const bool closed = p->green == SVH_GREEN_CLOSED_FORM && p->store.empty();
  if (closed) green_toeplitz_m0(p->K[0], p->K[1], p->K[2], p->T.data());
  free_tucker(p);
  dfree(p->d_zhat64);
  dfree(p->d_zhat32);
  dfree(p->d_g64);
  dfree(p->d_g32);
  dfree(p->d_g5_64);
  dfree(p->d_g5_32);
  dfree(p->d_gt64);
  dfree(p->d_gt32);
  p->diag_freq = -2;
  if (p->C == 5) {
    const svh_status st = setup_tensors5(p, s);
    if (st != SVH_OK) p->T.clear();
    return st;
  }
  const size_t Ht = folded_size(p);
  double *dT = nullptr, *t1 = nullptr;
  const size_t n1 = std::max((size_t)p->K[2] * p->K[1] * p->L[0],
                             (size_t)p->K[2] * (p->L[0] / 2 + 1) * (p->K[1] + p->L[1] / 2 + 1));
  const size_t n2 = (size_t)p->K[2] * p->L[1] * p->L[0];
  HIPCHK(hipMalloc(&p->d_zhat64, Ht * sizeof(double)));
  HIPCHK(hipMalloc(&p->d_zhat32, Ht * sizeof(float)));
  HIPCHK(hipMalloc(&p->d_g64, n2 * sizeof(double)));
  HIPCHK(hipMalloc(&p->d_g32, n2 * sizeof(float)));
  HIPCHK(hipMalloc(&dT, Kt * sizeof(double)));
  hipError_t e = hipMalloc(&t1, n1 * sizeof(double));
  if (closed) {
    if (e == hipSuccess) e = hipMemcpyAsync(dT, p->T.data(), Kt * sizeof(double), hipMemcpyHostToDevice, s);
  } else {
    // the Toeplitz tensor on the device, restored from the store (Algorithm 2)
    // or by quadrature; a host copy for the Tucker factorisation and the getters
    if (e == hipSuccess) e = p->store.empty() ? family_tables(p->K, 1, dT, s) : store_tables(p, 1, dT, s);
    if (e == hipSuccess) e = hipMemcpy(p->T.data(), dT, Kt * sizeof(double), hipMemcpyDeviceToHost);
  }
  // the x and y axes of the spectrum give the z-space kernel (direct z
  // step); the folded spectrum serves the z FFT step
  if (e == hipSuccess) e = launch_even_spectrum(p, dT, nullptr, t1, p->d_g64, s);
  if (e == hipSuccess) e = launch_folded_spectra(p, dT, 1, p->d_zhat64, t1, s);
  if (e == hipSuccess) e = launch_to_f32(p->d_zhat64, p->d_zhat32, Ht, s);
  if (e == hipSuccess) e = launch_to_f32(p->d_g64, p->d_g32, n2, s);
  if (e == hipSuccess && p->fused_r[0] > 0) {
    const size_t ng = p->dzset.size() * (size_t)p->L[0] * p->L[1];
    e = hipMalloc(&p->d_gt64, ng * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&p->d_gt32, ng * sizeof(float));
    if (e == hipSuccess) e = launch_gather_transposed(p, p->d_g64, p->d_gt64, s);
    if (e == hipSuccess) e = launch_to_f32(p->d_gt64, p->d_gt32, ng, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipFree(dT);
  if (t1) hipFree(t1);
  HIPCHK(e);
  return SVH_OK;
}

svh_status svh_set_green_method(svh_problem* p, int method) {
  if (!p) return SVH_EINVAL;
  if (method != SVH_GREEN_QUADRATURE && method != SVH_GREEN_CLOSED_FORM)
    return fail(p, SVH_EINVAL, "set_green_method: unknown method");
  p->green = method;
  return SVH_OK;
}

svh_status svh_get_family(const svh_problem* p, int family, double* T_host) {
  if (!p || !T_host || family < 0 || family >= kNFam) return SVH_EINVAL;
  const size_t Kt = (size_t)p->K[0] * p->K[1] * p->K[2];
  if (family == 0) {
    if (p->T.empty()) return SVH_ESTATE;
    std::memcpy(T_host, p->T.data(), Kt * sizeof(double));
    return SVH_OK;
  }
  if (p->C != 5) return SVH_EINVAL;
  if (p->Tf.size() != kNFam * Kt) return SVH_ESTATE;
  std::memcpy(T_host, p->Tf.data() + (size_t)family * Kt, Kt * sizeof(double));
  return SVH_OK;
}

svh_status svh_green_toeplitz(int Kx, int Ky, int Kz, double* T_host) {
  if (Kx < 1 || Ky < 1 || Kz < 1 || Kx > 4096 || Ky > 4096 || Kz > 4096 || !T_host) return SVH_EINVAL;
  green_toeplitz_m0(Kx, Ky, Kz, T_host);
  return SVH_OK;
}

svh_status svh_get_toeplitz(const svh_problem* p, double* T_host) {
  if (!p || !T_host) return SVH_EINVAL;
  if (p->T.empty()) return SVH_ESTATE;
  std::memcpy(T_host, p->T.data(), p->T.size() * sizeof(double));
  return SVH_OK;
}

svh_status svh_tucker_compress(svh_problem* p, double tol, int32_t* ranks_out, double* relerr_out) {
  if (!p) return SVH_EINVAL;
  if (!(tol >= 0)) return fail(p, SVH_EINVAL, "tucker_compress: tol must be >= 0");
  if (p->T.empty()) return fail(p, SVH_ESTATE, "tucker_compress: call svh_setup_tensors first");
  if (p->C == 5) {
    const size_t Kt = (size_t)p->K[0] * p->K[1] * p->K[2];
    free_tucker(p);
    double worst = 0;
    for (int f = 0; f < kNFam; ++f) {
      TuckerFactors tf;
      if (tucker_circulant(p->K, p->L, p->Tf.data() + f * Kt, kOdd[f], tol, tf) < 0)
        return fail(p, SVH_EINVAL, "tucker_compress: factorisation failed");
      DevTucker& t = p->tk5[f];
      for (int a = 0; a < 3; ++a) t.d[a] = tf.d[a];
      HIPCHK(upload(&t.core, tf.core.data(), tf.core.size()));
      for (int a = 0; a < 3; ++a) HIPCHK(upload(&t.F[a], tf.F[a].data(), tf.F[a].size()));
      if (p->d_qtab) {  // z-space factor at the distinct plane offsets (direct z step)
        const std::vector<double> Fz = zspace_factor(tf, p->L[2], p->dzset, kOdd[f][2] != 0);
        HIPCHK(upload(&t.Fz, Fz.data(), Fz.size()));
      }
      if (ranks_out)
        for (int a = 0; a < 3; ++a) ranks_out[3 * f + a] = tf.d[a];
      worst = std::max(worst, tf.relerr);
    }
    p->tucker = true;
    dfree(p->d_g5_64);
    dfree(p->d_g5_32);
    dfree(p->d_zhat64);
    dfree(p->d_zhat32);
    if (relerr_out) *relerr_out = worst;
    return SVH_OK;
  }
  TuckerFactors tf;
  if (tucker_even_circulant(p->K, p->L, p->T.data(), tol, tf) != 0)
    return fail(p, SVH_EINVAL, "tucker_compress: zero tensor");
  free_tucker(p);
  p->tk.d[0] = tf.d[0];
  p->tk.d[1] = tf.d[1];
  p->tk.d[2] = tf.d[2];
  HIPCHK(upload(&p->tk.core, tf.core.data(), tf.core.size()));
  for (int a = 0; a < 3; ++a) HIPCHK(upload(&p->tk.F[a], tf.F[a].data(), tf.F[a].size()));
  // z-space third factor: inverse z transform of F3 at offsets dz < Kz
  // (F3 columns are real and even in kz, so the transform is a cosine sum)
  {
    std::vector<int> dz(p->K[2]);
    for (int d = 0; d < p->K[2]; ++d) dz[d] = d;
    const std::vector<double> Fz = zspace_factor(tf, p->L[2], dz, false);
    HIPCHK(upload(&p->tk.Fz, Fz.data(), Fz.size()));
    if (!p->dzset.empty()) {
      const std::vector<double> Fzd = zspace_factor(tf, p->L[2], p->dzset, false);
      HIPCHK(upload(&p->tk.Fzd, Fzd.data(), Fzd.size()));
    }
  }
  p->tucker = true;
  dfree(p->d_zhat64);
  dfree(p->d_zhat32);
  dfree(p->d_g64);
  dfree(p->d_g32);
  dfree(p->d_gt64);
  dfree(p->d_gt32);
  if (ranks_out)
    for (int a = 0; a < 3; ++a) ranks_out[a] = tf.d[a];
  if (relerr_out) *relerr_out = tf.relerr;
  return SVH_OK;
}

size_t svh_workspace_bytes(const svh_problem* p, svh_prec prec, int nrhs) {
  if (!p || nrhs < 1) return 0;
  const size_t cs = prec == SVH_FP64 ? sizeof(double2) : sizeof(float2);
  const int cr = chunk_rhs(p, nrhs);
  size_t bf = 0;  // the fused path's need (AUTO may switch to it after svh_autotune)
  if (fused_eligible(p) && (p->zstep == SVH_ZSTEP_AUTO || p->zstep == SVH_ZSTEP_FUSED)) {
    const GeoT gt = make_geo_t(p, cs);
    bf = 2 * (((size_t)cr * p->C * p->zlist.size() * gt.pq * cs + 255) & ~(size_t)255);
    if (p->tucker) {
      const size_t ng = p->dzset.size() * (size_t)p->L[0] * p->L[1];
      bf += ((ng * (prec == SVH_FP64 ? sizeof(double) : sizeof(float)) + 255) & ~(size_t)255);
      bf += tucker_scratch_doubles(p) * sizeof(double);
    }
    bf += 1024;
    if (p->zstep == SVH_ZSTEP_FUSED) return bf;
  }
  size_t b = (size_t)cr * p->C * vec_bytes_AB(p, cs);
  if (p->tucker && p->C == 5) {
    const size_t gsz = use_zdirect(p) ? (size_t)kNFam * p->dzset.size() * p->L[0] * p->L[1]
                                      : (size_t)kNFam * folded_size(p);
    b += ((gsz * (prec == SVH_FP64 ? sizeof(double) : sizeof(float)) + 255) & ~(size_t)255) + 256;
    b += tucker_scratch_doubles5(p) * sizeof(double);
  } else if (p->tucker) {
    const size_t Lt = use_zdirect(p) ? (size_t)p->L[0] * p->L[1] * p->K[2] : folded_size(p);
    b += ((Lt * (prec == SVH_FP64 ? sizeof(double) : sizeof(float)) + 255) & ~(size_t)255);
    b += tucker_scratch_doubles(p) * sizeof(double);
  }
  return std::max(b + 1024, bf);
}

svh_status svh_matvec(svh_problem* p, svh_prec prec, int nrhs, const int32_t* freq_idx, const void* x,
                      void* y, void* ws, size_t ws_bytes, void* stream) {
  if (!p) return SVH_EINVAL;
  const long long ld = (long long)p->C * p->nvox;
  return svh::matvec_impl(p, prec, nrhs, freq_idx, x, ld, y, ld, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

svh_status svh_matvec_noalloc(svh_problem* p, svh_prec prec, int nrhs, const int32_t* freq_idx, const void* x,
                              void* y, void* stream) {
  if (!p) return SVH_EINVAL;
  if (nrhs < 1) return fail(p, SVH_EINVAL, "matvec_noalloc: bad arguments");
  if (p->prof) return fail(p, SVH_ESTATE, "matvec_noalloc: per-kernel profiling is enabled (it creates events)");
  const size_t need = svh_workspace_bytes(p, prec, nrhs);
  if (need > kScratchBytes)
    return fail(p, SVH_EINVAL, "matvec_noalloc: the batch needs " + std::to_string(need) +
                                   " bytes of workspace, more than the " + std::to_string(kScratchBytes) +
                                   " bytes of the static scratch array; use svh_matvec with a caller workspace");
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != p->device) return fail(p, SVH_EINVAL, "matvec_noalloc: the problem lives on another device");
  void* ws = nullptr;
  HIPCHK(scratch_address(dev, &ws));
  const long long ld = (long long)p->C * p->nvox;
  return svh::matvec_impl(p, prec, nrhs, freq_idx, x, ld, y, ld, ws, kScratchBytes,
                          static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace svh {
// Fused path: X pass (transposed store), fused y / z / inverse-y, inverse X
// pass; the z-space kernel of the occupied plane offsets comes from setup or
// from the Tucker factors.
static svh_status matvec_fused(svh_problem* p, svh_prec prec, int nrhs, const int32_t* freq_idx, const void* x,
                               long long ldx, void* y, long long ldy, void* ws, size_t ws_bytes, hipStream_t s,
                               int cr) {
  const bool dbl = prec == SVH_FP64;
  const size_t cs = dbl ? sizeof(double2) : sizeof(float2);
  auto align = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const GeoT gt = make_geo_t(p, cs);
  const size_t buf = align((size_t)cr * p->C * p->zlist.size() * gt.pq * cs);
  char* w = static_cast<char*>(ws);
  char* A = w;
  char* O = w + buf;
  const void* gk = dbl ? (const void*)p->d_gt64 : (const void*)p->d_gt32;
  std::vector<hipEvent_t> evs;
  if (p->prof) {
    const int nchunk = (nrhs + cr - 1) / cr;
    for (int i = 0; i < 8 * nchunk; ++i) {
      hipEvent_t e;
      if (!p->prof_pool.empty()) {
        e = p->prof_pool.back();
        p->prof_pool.pop_back();
      } else {
        HIPCHK(hipEventCreate(&e));
      }
      evs.push_back(e);
    }
    HIPCHK(hipEventRecord(evs[0], s));
  }
  if (p->tucker) {
    char* zb = O + buf;
    const size_t ng = p->dzset.size() * (size_t)p->L[0] * p->L[1];
    double* V = reinterpret_cast<double*>(zb + align(ng * (dbl ? 8 : 4)));
    double* Wt = V + (size_t)p->L[0] * p->tk.d[1] * p->tk.d[2];
    if (reinterpret_cast<char*>(Wt + (size_t)p->L[0] * p->L[1] * p->tk.d[2]) > w + ws_bytes)
      return fail(p, SVH_EINVAL, "matvec: workspace too small");
    HIPCHK(launch_tucker_rebuild_rows(p, p->tk, p->tk.Fzd, (int)p->dzset.size(), !dbl, zb, V, Wt, s, true));
    gk = zb;
  } else if (!gk) {
    return fail(p, SVH_ESTATE, "matvec: no z-space kernel");
  }
  if (p->prof) HIPCHK(hipEventRecord(evs[1], s));
  const char* xb = static_cast<const char*>(x);
  for (int r0 = 0; r0 < nrhs; r0 += cr) {
    const int nr = std::min(cr, nrhs - r0);
    hipEvent_t* ev = nullptr;
    if (p->prof) {
      ev = &evs[8 * (r0 / cr) + 2];
      if (r0 > 0) {
        HIPCHK(hipEventRecord(evs[8 * (r0 / cr)], s));
        HIPCHK(hipEventRecord(evs[8 * (r0 / cr) + 1], s));
      }
    }
    EpiParams ep;
    ep.C = p->C;
    ep.K = p->nvox;
    ep.vec0 = 0;
    ep.ldx = ldx;
    ep.ldy = ldy;
    for (int i = 0; i < kMaxVecsPerChunk; ++i) ep.fidx[i] = -1;
    for (int i = 0; i < nr; ++i) ep.fidx[i] = freq_idx[r0 + i];
    const char* xc = xb + (size_t)r0 * ldx * cs;
    char* yc = static_cast<char*>(y) + (size_t)r0 * ldy * cs;
    hipError_t e = dbl ? launch_matvec_chunk_fused<double>(p, nr * p->C, ep, xc, yc, A, O, gk, s, ev)
                       : launch_matvec_chunk_fused<float>(p, nr * p->C, ep, xc, yc, A, O, gk, s, ev);
    HIPCHK(e);
  }
  for (size_t i = 0; i < evs.size(); i += 8)
    p->prof_events.push_back(std::vector<hipEvent_t>(evs.begin() + i, evs.begin() + i + 8));
  return SVH_OK;
}

svh_status matvec_impl(svh_problem* p, svh_prec prec, int nrhs, const int32_t* freq_idx, const void* x,
                       long long ldx, void* y, long long ldy, void* ws, size_t ws_bytes, hipStream_t s) {
  if (nrhs < 1 || !freq_idx || !x || !y || !ws) return fail(p, SVH_EINVAL, "matvec: bad arguments");
  if (prec != SVH_FP64 && prec != SVH_FP32) return fail(p, SVH_EINVAL, "matvec: bad precision");
  if (!p->tucker && !p->d_zhat64 && !p->d_g5_64) return fail(p, SVH_ESTATE, "matvec: call svh_setup_tensors first");
  for (int r = 0; r < nrhs; ++r) {
    if (freq_idx[r] < -1 || freq_idx[r] >= p->nfreq)
      return fail(p, SVH_EINVAL, "matvec: frequency index out of range (set the material first)");
  }
  const size_t need = svh_workspace_bytes(p, prec, nrhs);
  if (ws_bytes < need) return fail(p, SVH_EINVAL, "matvec: workspace too small");
  const bool dbl = prec == SVH_FP64;
  const size_t cs = dbl ? sizeof(double2) : sizeof(float2);
  const long long ck = (long long)p->C * p->nvox;
  if (ldx < ck || ldy < ck) return fail(p, SVH_EINVAL, "matvec: stride below one vector");
  // overlap check of x and y (whole strided extents)
  const char* xb = static_cast<const char*>(x);
  const char* yb = static_cast<const char*>(y);
  const size_t xext = ((size_t)(nrhs - 1) * ldx + ck) * cs;
  const size_t yext = ((size_t)(nrhs - 1) * ldy + ck) * cs;
  if (xb < yb + yext && yb < xb + xext) return fail(p, SVH_EINVAL, "matvec: x and y overlap");
  char* w = static_cast<char*>(ws);
  auto align = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const int cr = chunk_rhs(p, nrhs);
  const size_t nzp = p->zlist.size();
  if (use_fused(p, prec)) return matvec_fused(p, prec, nrhs, freq_idx, x, ldx, y, ldy, ws, ws_bytes, s, cr);
  const Geo geo = make_geo(p, cs);
  const size_t Abytes = align((size_t)cr * p->C * nzp * geo.pa * cs);
  const size_t Bbytes = (size_t)cr * p->C * nzp * geo.pb * cs;
  char* A = w;
  char* B = w + Abytes;
  const bool zdirect = use_zdirect(p);
  const void* zhat = !zdirect ? (dbl ? (const void*)p->d_zhat64 : (const void*)p->d_zhat32)
                     : p->C == 5 ? (dbl ? (const void*)p->d_g5_64 : (const void*)p->d_g5_32)
                                 : (dbl ? (const void*)p->d_g64 : (const void*)p->d_g32);
  std::vector<hipEvent_t> evs;
  if (p->prof) {
    const int nchunk = (nrhs + cr - 1) / cr;
    for (int i = 0; i < 8 * nchunk; ++i) {
      hipEvent_t e;
      if (!p->prof_pool.empty()) {
        e = p->prof_pool.back();
        p->prof_pool.pop_back();
      } else {
        HIPCHK(hipEventCreate(&e));
      }
      evs.push_back(e);
    }
    HIPCHK(hipEventRecord(evs[0], s));
  }
  const int hx = p->L[0] / 2 + 1, hy = p->L[1] / 2 + 1, hz = p->L[2] / 2 + 1;
  if (p->tucker && p->C == 5) {
    // restore the seven families' z-space kernels (direct z step) or folded
    // spectra (z FFT step) one after another
    char* zb = B + align(Bbytes);
    const int nd = (int)p->dzset.size();
    const size_t rows = zdirect ? (size_t)nd * p->L[0] * p->L[1] : folded_size(p);
    const size_t gbytes = align(kNFam * rows * (dbl ? 8 : 4));
    double* V = reinterpret_cast<double*>(zb + gbytes);
    for (int f = 0; f < kNFam; ++f) {
      const DevTucker& t = p->tk5[f];
      double* Wt = V + (size_t)p->L[0] * t.d[1] * t.d[2];
      if (reinterpret_cast<char*>(Wt + (size_t)p->L[0] * p->L[1] * t.d[2]) > w + ws_bytes)
        return fail(p, SVH_EINVAL, "matvec: workspace too small");
      void* out = zb + f * rows * (dbl ? 8 : 4);
      if (zdirect) HIPCHK(launch_tucker_rebuild_rows(p, t, t.Fz, nd, !dbl, out, V, Wt, s));
      else HIPCHK(launch_tucker_box(hx, hy, hz, t, t.F[2], !dbl, out, V, Wt, s));
    }
    zhat = zb;
  } else if (p->tucker && !zdirect) {
    char* zb = B + align(Bbytes);
    double* V = reinterpret_cast<double*>(zb + align(folded_size(p) * (dbl ? 8 : 4)));
    double* Wt = V + (size_t)p->L[0] * p->tk.d[1] * p->tk.d[2];
    if (reinterpret_cast<char*>(Wt + (size_t)p->L[0] * p->L[1] * p->tk.d[2]) > w + ws_bytes)
      return fail(p, SVH_EINVAL, "matvec: workspace too small");
    HIPCHK(launch_tucker_box(hx, hy, hz, p->tk, p->tk.F[2], !dbl, zb, V, Wt, s));
    zhat = zb;
  } else if (p->tucker) {
    char* zb = B + align(Bbytes);
    const size_t Lt = (size_t)p->L[0] * p->L[1] * (zdirect ? p->K[2] : p->L[2]);
    double* V = reinterpret_cast<double*>(zb + align(Lt * (dbl ? 8 : 4)));
    double* Wt = V + (size_t)p->L[0] * p->tk.d[1] * p->tk.d[2];
    if (reinterpret_cast<char*>(Wt + (size_t)p->L[0] * p->L[1] * p->tk.d[2]) > w + ws_bytes)
      return fail(p, SVH_EINVAL, "matvec: workspace too small");
    if (zdirect && p->d_qtab)  // only the distinct plane offsets, indexed by slot
      HIPCHK(launch_tucker_rebuild_rows(p, p->tk, p->tk.Fzd, (int)p->dzset.size(), !dbl, zb, V, Wt, s));
    else
      HIPCHK(launch_tucker_rebuild(p, !dbl, zdirect, zb, V, Wt, s));
    zhat = zb;
  } else if (!zhat) {
    return fail(p, SVH_ESTATE, "matvec: no spectrum");
  }
  if (p->prof) HIPCHK(hipEventRecord(evs[1], s));
  for (int r0 = 0; r0 < nrhs; r0 += cr) {
    const int nr = std::min(cr, nrhs - r0);
    hipEvent_t* ev = nullptr;
    if (p->prof) {
      ev = &evs[8 * (r0 / cr) + 2];
      if (r0 > 0) {
        HIPCHK(hipEventRecord(evs[8 * (r0 / cr)], s));
        HIPCHK(hipEventRecord(evs[8 * (r0 / cr) + 1], s));
      }
    }
    EpiParams ep;
    ep.C = p->C;
    ep.K = p->nvox;
    ep.vec0 = 0;
    ep.ldx = ldx;
    ep.ldy = ldy;
    ep.zslot = p->C == 3 && p->tucker && zdirect && p->d_qtab != nullptr;
    for (int i = 0; i < kMaxVecsPerChunk; ++i) ep.fidx[i] = -1;
    for (int i = 0; i < nr; ++i) ep.fidx[i] = freq_idx[r0 + i];
    const char* xc = xb + (size_t)r0 * ldx * cs;
    char* yc = static_cast<char*>(y) + (size_t)r0 * ldy * cs;
    hipError_t e = dbl ? launch_matvec_chunk<double>(p, nr * p->C, ep, xc, yc, A, B, zhat, s, ev)
                       : launch_matvec_chunk<float>(p, nr * p->C, ep, xc, yc, A, B, zhat, s, ev);
    if (e == hipErrorInvalidConfiguration)
      return fail(p, SVH_EINVAL, "matvec: the z step of this grid needs more LDS per block than the device has");
    HIPCHK(e);
  }
  for (size_t i = 0; i < evs.size(); i += 8)
    p->prof_events.push_back(std::vector<hipEvent_t>(evs.begin() + i, evs.begin() + i + 8));
  return SVH_OK;
}
}  // namespace svh

extern "C" {

svh_status svh_autotune(svh_problem* p, svh_prec prec, int nrhs, const int32_t* freq_idx, const void* x, void* y,
                        void* ws, size_t ws_bytes, void* stream, double* ms_out) {
  if (!p) return SVH_EINVAL;
  if (prec != SVH_FP64 && prec != SVH_FP32) return fail(p, SVH_EINVAL, "autotune: bad precision");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool was_prof = p->prof;
  Tune best;
  double best_ms[4] = {1e30, 1e30, 1e30, 1e30};
  svh_status st = SVH_OK;
  p->prof = true;
  // candidates: persistent grid multiplier x column width of the y passes
  for (int c = 0; c < 8 && st == SVH_OK; ++c) {
    const int mult = kTuneCandidates[c % 4], shift = c / 4;
    for (int i = 0; i < 4; ++i) p->tune[prec].grid_mult[i] = mult;
    p->tune[prec].ycols_shift[0] = p->tune[prec].ycols_shift[1] = shift;
    st = svh_matvec(p, prec, nrhs, freq_idx, x, y, ws, ws_bytes, stream);  // warm-up
    double ms[SVH_NPROF];
    int n = 0;
    if (st == SVH_OK) st = svh_profile_read(p, ms, &n);
    for (int rep = 0; rep < 2 && st == SVH_OK; ++rep)
      st = svh_matvec(p, prec, nrhs, freq_idx, x, y, ws, ws_bytes, stream);
    if (st == SVH_OK) st = svh_profile_read(p, ms, &n);
    if (st != SVH_OK) break;
    for (int i = 0; i < 4; ++i) {
      const double t = ms[1 + (i == 0 ? 0 : i == 1 ? 1 : i == 2 ? 3 : 4)];  // X, Y, Yi, Xi slots
      if (t < best_ms[i]) {
        best_ms[i] = t;
        best.grid_mult[i] = mult;
        if (i == 1) best.ycols_shift[0] = shift;
        if (i == 2) best.ycols_shift[1] = shift;
      }
    }
  }
  p->tune[prec] = best;
  if (st == SVH_OK && p->zstep == SVH_ZSTEP_AUTO && fused_eligible(p)) {
    // AUTO: keep the faster of the separate passes and the fused step
    double tot[2] = {0, 0};
    for (int v = 0; v < 2 && st == SVH_OK; ++v) {
      p->auto_fused[prec] = v == 1;
      st = svh_matvec(p, prec, nrhs, freq_idx, x, y, ws, ws_bytes, stream);  // warm-up
      double ms[SVH_NPROF];
      int n = 0;
      if (st == SVH_OK) st = svh_profile_read(p, ms, &n);
      for (int rep = 0; rep < 2 && st == SVH_OK; ++rep)
        st = svh_matvec(p, prec, nrhs, freq_idx, x, y, ws, ws_bytes, stream);
      if (st == SVH_OK) st = svh_profile_read(p, ms, &n);
      for (int i = 0; i < SVH_NPROF && st == SVH_OK; ++i) tot[v] += ms[i];
    }
    p->auto_fused[prec] = st == SVH_OK && tot[1] < tot[0];
  }
  p->prof = was_prof;
  if (st != SVH_OK) return st;
  HIPCHK(hipStreamSynchronize(s));
  if (ms_out) {
    double ms[SVH_NPROF];
    int n = 0;
    p->prof = true;
    st = svh_matvec(p, prec, nrhs, freq_idx, x, y, ws, ws_bytes, stream);
    if (st == SVH_OK) st = svh_profile_read(p, ms, &n);
    p->prof = was_prof;
    if (st != SVH_OK) return st;
    double tot = 0;
    for (int i = 0; i < SVH_NPROF; ++i) tot += ms[i];
    *ms_out = tot;
  }
  return SVH_OK;
}

svh_status svh_set_zstep(svh_problem* p, int mode) {
  if (!p) return SVH_EINVAL;
  if (mode != SVH_ZSTEP_AUTO && mode != SVH_ZSTEP_FFT && mode != SVH_ZSTEP_DIRECT && mode != SVH_ZSTEP_FUSED)
    return fail(p, SVH_EINVAL, "set_zstep: unknown mode");
  if (mode == SVH_ZSTEP_FUSED && (p->C != 3 || p->fused_r[0] <= 0 || p->fused_r[1] <= 0 ||
                                  p->zlist.size() > (size_t)kMaxDirectPlanes))
    return fail(p, SVH_EINVAL, "set_zstep: the fused step needs basis 3 and at most 32 occupied planes with at "
                               "most 64 distinct plane offsets");
  if (mode == SVH_ZSTEP_DIRECT && (int)p->zlist.size() > kMaxDirectPlanes)
    return fail(p, SVH_EINVAL, "set_zstep: direct z sum supports at most 32 occupied planes");
  if (mode == SVH_ZSTEP_DIRECT && p->C == 5 && !p->d_qtab)
    return fail(p, SVH_EINVAL, "set_zstep: the five-component direct z sum supports at most 64 distinct plane "
                               "offsets");
  p->zstep = mode;
  return SVH_OK;
}

svh_status svh_profile_enable(svh_problem* p, int enable) {
  if (!p) return SVH_EINVAL;
  p->prof = enable != 0;
  return SVH_OK;
}

svh_status svh_profile_read(svh_problem* p, double* ms_out, int* ncalls_out) {
  if (!p || !ms_out) return SVH_EINVAL;
  for (int i = 0; i < SVH_NPROF; ++i) ms_out[i] = 0;
  int n = 0;
  for (auto& set : p->prof_events) {
    HIPCHK(hipEventSynchronize(set[7]));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, set[0], set[1]));
    ms_out[0] += ms;
    for (int k = 0; k < 5; ++k) {
      HIPCHK(hipEventElapsedTime(&ms, set[2 + k], set[3 + k]));
      ms_out[1 + k] += ms;
    }
    for (hipEvent_t e : set) p->prof_pool.push_back(e);
    ++n;
  }
  p->prof_events.clear();
  if (ncalls_out) *ncalls_out = n;
  return SVH_OK;
}

const char* svh_last_error(const svh_problem* p) {
  if (!p) return "null problem";
  return p->err.c_str();
}

void svh_destroy(svh_problem* p) {
  if (!p) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(p->device);
  dfree(p->d_xrow);
  dfree(p->d_zlist);
  dfree(p->d_zslot);
  for (int a = 0; a < 3; ++a) {
    dfree(p->d_tw64[a]);
    dfree(p->d_tw32[a]);
  }
  dfree(p->d_sconv64);
  dfree(p->d_sconv32);
  dfree(p->d_cdiag64);
  dfree(p->d_cdiag32);
  dfree(p->d_zhat64);
  dfree(p->d_zhat32);
  dfree(p->d_g64);
  dfree(p->d_g32);
  dfree(p->d_g5_64);
  dfree(p->d_g5_32);
  dfree(p->d_gt64);
  dfree(p->d_gt32);
  dfree(p->d_twp64);
  dfree(p->d_twp32);
  dfree(p->d_qtab);
  free_tucker(p);
  svh::free_solver(p);
  for (auto& set : p->prof_events)
    for (hipEvent_t e : set) (void)hipEventDestroy(e);
  for (hipEvent_t e : p->prof_pool) (void)hipEventDestroy(e);
  (void)hipSetDevice(cur);
  delete p;
}

}  // extern "C"
