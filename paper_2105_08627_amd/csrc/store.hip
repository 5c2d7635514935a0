// Toeplitz store (Algorithm 2, Sec. II.B.1): the unit-voxel integral tables of
// a large domain, Tucker-compressed once (installation) and written to a file;
// at setup the tables of a problem's grid are restored from the factors'
// leading rows (the trim of Algorithm 2) on the matrix cores.  The (dx)^5
// scale of Algorithm 2 is not applied to the tables: with the total-current
// basis normalisation it combines to the factor j w mu0 dx that the product
// applies per frequency.
//
// File layout (little endian): "SVHTSTOR", int32 version = 1, int32 nfam,
// int32 K[3], double tol; then per family int32 d[3], double relerr, the core
// (d3 d2 d1 doubles, [c][b][a]) and the factors F1 (K1 x d1), F2, F3 ([k][c]).
#include <cstdio>
#include <cstring>
#include <memory>

#include "svh_internal.h"

namespace svh {

namespace {
constexpr char kMagic[8] = {'S', 'V', 'H', 'T', 'S', 'T', 'O', 'R'};

struct FileCloser {
  void operator()(FILE* f) const {
    if (f) fclose(f);
  }
};
using FilePtr = std::unique_ptr<FILE, FileCloser>;

template <typename T> bool put(FILE* f, const T* v, size_t n) { return fwrite(v, sizeof(T), n, f) == n; }
template <typename T> bool get(FILE* f, T* v, size_t n) { return fread(v, sizeof(T), n, f) == n; }
}  // namespace

int read_store(const char* path, int K[3], std::vector<TuckerFactors>& fam, std::string& err) {
  FilePtr f(fopen(path, "rb"));
  if (!f) {
    err = std::string("cannot open ") + path;
    return -1;
  }
  char magic[8];
  int32_t ver = 0, nfam = 0, k[3];
  double tol = 0;
  if (!get(f.get(), magic, 8) || std::memcmp(magic, kMagic, 8) != 0 || !get(f.get(), &ver, 1) || ver != 1 ||
      !get(f.get(), &nfam, 1) || (nfam != 1 && nfam != kNFam) || !get(f.get(), k, 3) || !get(f.get(), &tol, 1)) {
    err = "not a Toeplitz store file";
    return -1;
  }
  for (int a = 0; a < 3; ++a) {
    if (k[a] < 1 || k[a] > 4096) {
      err = "bad store domain";
      return -1;
    }
    K[a] = k[a];
  }
  fam.assign(nfam, TuckerFactors());
  for (int i = 0; i < nfam; ++i) {
    TuckerFactors& t = fam[i];
    int32_t d[3];
    if (!get(f.get(), d, 3) || !get(f.get(), &t.relerr, 1)) {
      err = "truncated store file";
      return -1;
    }
    for (int a = 0; a < 3; ++a) {
      if (d[a] < 1 || d[a] > K[a]) {
        err = "bad store ranks";
        return -1;
      }
      t.d[a] = d[a];
    }
    t.core.resize((size_t)d[0] * d[1] * d[2]);
    bool ok = get(f.get(), t.core.data(), t.core.size());
    for (int a = 0; a < 3 && ok; ++a) {
      t.F[a].resize((size_t)K[a] * d[a]);
      ok = get(f.get(), t.F[a].data(), t.F[a].size());
    }
    if (!ok) {
      err = "truncated store file";
      return -1;
    }
  }
  return 0;
}

static hipError_t restore_tables(const std::vector<TuckerFactors>& store, const int K[3], int nfam, double* d_out,
                                 hipStream_t s) {
  const int n1 = K[0], n2 = K[1], n3 = K[2];
  const size_t Kt = (size_t)n1 * n2 * n3;
  hipError_t e = hipSuccess;
  for (int f = 0; f < nfam && e == hipSuccess; ++f) {
    const TuckerFactors& tf = store[f];
    DevTucker t;
    for (int a = 0; a < 3; ++a) t.d[a] = tf.d[a];
    double *V = nullptr, *W = nullptr;
    e = hipMalloc(&t.core, tf.core.size() * sizeof(double));
    for (int a = 0; a < 3 && e == hipSuccess; ++a) e = hipMalloc(&t.F[a], tf.F[a].size() * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&V, (size_t)n1 * t.d[1] * t.d[2] * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&W, (size_t)n1 * n2 * t.d[2] * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(t.core, tf.core.data(), tf.core.size() * sizeof(double), hipMemcpyHostToDevice);
    for (int a = 0; a < 3 && e == hipSuccess; ++a)
      e = hipMemcpy(t.F[a], tf.F[a].data(), tf.F[a].size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_tucker_box(n1, n2, n3, t, t.F[2], false, d_out + f * Kt, V, W, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(V);
    hipFree(W);
    hipFree(t.core);
    for (int a = 0; a < 3; ++a) hipFree(t.F[a]);
  }
  return e;
}

hipError_t store_tables(const svh_problem* p, int nfam, double* d_out, hipStream_t s) {
  return restore_tables(p->store, p->K, nfam, d_out, s);
}

}  // namespace svh

using namespace svh;

extern "C" {

svh_status svh_toeplitz_store_build(int Kx, int Ky, int Kz, int nfam, double tol, const char* path, void* stream,
                                    double* relerr_out) {
  if (Kx < 1 || Ky < 1 || Kz < 1 || Kx > 4096 || Ky > 4096 || Kz > 4096 || (nfam != 1 && nfam != kNFam) ||
      !(tol >= 0) || !path)
    return SVH_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int K[3] = {Kx, Ky, Kz};
  const size_t Kt = (size_t)Kx * Ky * Kz;
  double* d = nullptr;
  hipError_t e = hipMalloc(&d, (size_t)nfam * Kt * sizeof(double));
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? SVH_ENOMEM : SVH_EHIP;
  std::vector<double> T((size_t)nfam * Kt);
  e = family_tables(K, nfam, d, s);
  if (e == hipSuccess) e = hipMemcpy(T.data(), d, T.size() * sizeof(double), hipMemcpyDeviceToHost);
  hipFree(d);
  if (e != hipSuccess) return SVH_EHIP;
  FilePtr f(fopen(path, "wb"));
  if (!f) return SVH_EINVAL;
  const int32_t ver = 1, nf = nfam, k[3] = {Kx, Ky, Kz};
  bool ok = put(f.get(), kMagic, 8) && put(f.get(), &ver, 1) && put(f.get(), &nf, 1) && put(f.get(), k, 3) &&
            put(f.get(), &tol, 1);
  double worst = 0;
  for (int i = 0; i < nfam && ok; ++i) {
    TuckerFactors tf;
    if (tucker_plain(K, T.data() + i * Kt, tol, tf) < 0) return SVH_EINVAL;
    const int32_t dd[3] = {tf.d[0], tf.d[1], tf.d[2]};
    ok = put(f.get(), dd, 3) && put(f.get(), &tf.relerr, 1) && put(f.get(), tf.core.data(), tf.core.size());
    for (int a = 0; a < 3 && ok; ++a) ok = put(f.get(), tf.F[a].data(), tf.F[a].size());
    worst = std::max(worst, tf.relerr);
  }
  if (!ok) return SVH_EINVAL;
  if (relerr_out) *relerr_out = worst;
  return SVH_OK;
}

svh_status svh_green_tables(int Kx, int Ky, int Kz, int nfam, double* T_dev, void* stream) {
  if (Kx < 1 || Ky < 1 || Kz < 1 || Kx > 4096 || Ky > 4096 || Kz > 4096 || (nfam != 1 && nfam != kNFam) || !T_dev)
    return SVH_EINVAL;
  const int K[3] = {Kx, Ky, Kz};
  hipStream_t s = static_cast<hipStream_t>(stream);
  return family_tables(K, nfam, T_dev, s) == hipSuccess && hipStreamSynchronize(s) == hipSuccess ? SVH_OK
                                                                                                 : SVH_EHIP;
}

svh_status svh_toeplitz_store_restore(const char* path, int Kx, int Ky, int Kz, int nfam, double* T_dev,
                                      void* stream) {
  if (!path || Kx < 1 || Ky < 1 || Kz < 1 || nfam < 1 || !T_dev) return SVH_EINVAL;
  int K[3];
  std::vector<TuckerFactors> fam;
  std::string err;
  if (read_store(path, K, fam, err) != 0) return SVH_EINVAL;
  if (Kx > K[0] || Ky > K[1] || Kz > K[2] || nfam > (int)fam.size()) return SVH_EINVAL;
  const int Kp[3] = {Kx, Ky, Kz};
  return restore_tables(fam, Kp, nfam, T_dev, static_cast<hipStream_t>(stream)) == hipSuccess ? SVH_OK : SVH_EHIP;
}

svh_status svh_set_toeplitz_store(svh_problem* p, const char* path) {
  if (!p) return SVH_EINVAL;
  if (!path) {
    p->store.clear();
    return SVH_OK;
  }
  int K[3];
  std::vector<TuckerFactors> fam;
  if (read_store(path, K, fam, p->err) != 0) return SVH_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (K[a] < p->K[a]) {
      p->err = "set_toeplitz_store: the stored domain is smaller than the grid";
      return SVH_EINVAL;
    }
  if (p->C == 5 && (int)fam.size() < kNFam) {
    p->err = "set_toeplitz_store: the piecewise-linear basis needs all seven integral families";
    return SVH_EINVAL;
  }
  for (int a = 0; a < 3; ++a) p->store_K[a] = K[a];
  p->store = std::move(fam);
  return SVH_OK;
}

}  // extern "C"
