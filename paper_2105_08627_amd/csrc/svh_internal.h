// Internal declarations of the SVH library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/svh.h"
#include "host_math.h"

namespace svh {

constexpr double kMu0 = 4.0e-7 * 3.14159265358979323846;  // H/m (mu = mu0, Sec. II.A)
constexpr int kMaxVecsPerChunk = 320;  // component vectors per pass launch (64 RHS of five components)
constexpr int kMaxStages = 8;
constexpr int kMaxDirectPlanes = 32;  // direct z sum when at most this many planes are occupied
// Piecewise-linear basis (eqs. 4-8): seven voxel-pair integral families
// M0, M1x, M1y, M1z, M2x, M2y, M2z; the M1 family of axis a is odd along a.
constexpr int kNFam = 7;
constexpr int kMaxDz5 = 64;  // distinct plane offsets of the coupled direct z step

// Mixed-radix Stockham plan: L = prod r[s], radices in {8, 4, 2, 3}.
struct FftPlan {
  int L = 0;
  int ns = 0;
  int r[kMaxStages] = {0};
  int tp = 0;  // threads per pencil = min_s L / r[s]
};
bool make_plan(int L, FftPlan& p);
FftPlan reversed(const FftPlan& p);
bool supported_length(int L);

// Device-side Tucker representation of one spectrum.
struct DevTucker {
  int d[3] = {0, 0, 0};
  double* core = nullptr;  // [c][b][a]
  double* F[3] = {nullptr, nullptr, nullptr};  // [k][c]
  double* Fz = nullptr;  // [dz][c], dz < Kz: inverse z transform of F[2] (z-space factor)
  double* Fzd = nullptr; // [slot][c]: the same at the occupied plane offsets only
};

// Occupancy of 64 consecutive x positions of one grid row: bit b set when
// voxel x = 64 w + b is non-empty; base = compact index of the first such
// voxel.  Voxels are numbered z-, y-, x-major, so the voxel at bit b has the
// compact index base + (set bits below b).
struct alignas(16) XRowWord {
  unsigned long long bits;
  int base;
  int pad;
};

// Per-call kernel parameters of the final (x-inverse) pass.
struct EpiParams {
  int C;              // components per right-hand side
  int K;              // non-empty voxels
  int vec0;           // first component-vector of this chunk
  long long ldx, ldy; // element stride between right-hand sides of x and y
  int fidx[kMaxVecsPerChunk];  // frequency slot per RHS of the chunk (-1 = bare)
  bool zslot = false;          // direct z step: kernel rows indexed by offset slot (dzset), not by offset
};

// Strides (in complex elements) of the intermediate buffers
// A[vec][plane][y < Ky][x < Lx] and B[vec][plane][ky < Ly][x < Lx]: rows and
// planes are padded off powers of two so that the rows a column pass touches
// spread over memory channels instead of aliasing onto one.
struct Geo {
  int rp;          // row pitch
  long long pa;    // plane stride of A
  long long pb;    // plane stride of B
};

// Transposed buffers of the fused path: element (vec, plane, kx, y) at
// (vec * nzp + plane) * pq + kx * cp + y.
struct GeoT {
  int cp;          // column pitch (>= Ky)
  long long pq;    // plane stride
};

// Launch choices of the FFT passes, picked by svh_autotune per precision.
// grid_mult[i] for pass i in {X, Y, Yi, Xi}: the persistent launch uses
// (resident blocks per CU x CUs x grid_mult) blocks; 0 = one block per item.
constexpr int kTuneCandidates[4] = {1, 2, 4, 0};
struct Tune {
  int grid_mult[4] = {1, 1, 1, 1};
  int ycols_shift[2] = {0, 0};  // Y, Yi: columns per block = widest >> shift
};

}  // namespace svh

struct svh_problem {
  int K[3] = {0, 0, 0};
  int L[3] = {0, 0, 0};
  double dx = 0;
  int basis = 3;
  int C = 3;
  int nvox = 0;
  int device = 0;
  int ncu = 256;  // compute units of the device
  int max_lds = 65536;  // bytes of LDS one block may use on the device
  std::vector<int32_t> vidx;       // dense -> compact index or -1, [z][y][x]
  std::vector<int32_t> zlist;      // occupied z planes
  std::vector<int32_t> zslot;      // z -> plane slot or -1 (size L[2])
  svh::XRowWord* d_xrow = nullptr;      // [plane slot][y][x / 64] occupancy words of the occupied planes
  int xrow_words = 0;              // words per row, ceil(Kx / 64)
  int32_t* d_zlist = nullptr;
  int32_t* d_zslot = nullptr;
  svh::FftPlan plan[3];
  double2* d_tw64[3] = {nullptr, nullptr, nullptr};  // e^{-2 pi i m / L}
  float2* d_tw32[3] = {nullptr, nullptr, nullptr};
  // material
  int nfreq = 0;
  std::vector<std::complex<double>> sconv;  // j w mu0 dx per frequency
  double2* d_sconv64 = nullptr;             // [nfreq]
  float2* d_sconv32 = nullptr;
  double2* d_cdiag64 = nullptr;  // [nfreq][K] c / dx
  float2* d_cdiag32 = nullptr;
  // tensors
  std::vector<double> T;        // Toeplitz tensor, host [Kz][Ky][Kx]
  // piecewise-linear basis (C = 5): family tables (host, [f][Kz][Ky][Kx];
  // f = 0 is T), the distinct plane offsets |z_i - z_j| of the occupied planes,
  // the (row, column) -> offset-slot codes of the coupled z step and the
  // z-space kernels [f][slot][Ly][Lx] (for M1x, M1y the coefficient of j)
  std::vector<double> Tf;
  std::vector<int32_t> dzset;
  uint8_t* d_qtab = nullptr;    // [32][32]: slot | 0x80 when z_j < z_i
  double* d_g5_64 = nullptr;
  float* d_g5_32 = nullptr;
  svh::DevTucker tk5[svh::kNFam];
  // spectra of the circulants (real; j times this for M1x, M1y, M1z), folded
  // to k_a <= L_a / 2 per axis: [f][kz][ky][kx], one family (basis 3) or seven
  double* d_zhat64 = nullptr;
  float* d_zhat32 = nullptr;
  double* d_g64 = nullptr;      // dense z-space kernel [Kz][Ly][Lx] (real)
  float* d_g32 = nullptr;
  // fused y / z / inverse-y path: z-space kernel at the occupied plane
  // offsets, transposed in (x, y): [slot][kx][ky]; frequency phases per
  // precision (index SVH_FP64, SVH_FP32) and twiddles of length Ly / phases
  double* d_gt64 = nullptr;
  float* d_gt32 = nullptr;
  int fused_r[2] = {0, 0};
  int fused2_r = 0;  // phases of the resident-kernel fused step (FP32), 0: not applicable
  bool auto_fused[2] = {false, false};  // AUTO mode: the autotuner timed FUSED faster
  double2* d_twp64 = nullptr;
  float2* d_twp32 = nullptr;
  int zstep = 0;                // SVH_ZSTEP_AUTO / _FFT / _DIRECT / _FUSED
  int green = 0;                // SVH_GREEN_QUADRATURE (device) / SVH_GREEN_CLOSED_FORM (host, M0)
  // Toeplitz store (Algorithm 2): Tucker factors of the tables on a large
  // unit-voxel domain, read by svh_set_toeplitz_store; empty = not used
  int store_K[3] = {0, 0, 0};
  std::vector<svh::TuckerFactors> store;
  svh::Tune tune[2];            // per precision (SVH_FP64, SVH_FP32)
  bool tucker = false;
  svh::DevTucker tk;
  std::vector<std::complex<double>> cdiag_host;  // [nfreq][K] c / dx
  // saddle system (eq. 7) and ports
  bool topo_built = false;
  svh::Topology topo;
  int nports = 0;
  std::vector<char> dirichlet;          // per node
  std::vector<double> bport_host;       // [nports][C*K] port vectors A_{q+}^T 1
  std::vector<std::vector<int>> port_plus;  // + terminal nodes per port
  int32_t *d_cptr = nullptr, *d_crow = nullptr, *d_rptr = nullptr, *d_rcol = nullptr;
  double *d_cval = nullptr, *d_rval = nullptr;
  uint8_t* d_free = nullptr;
  double* d_bport = nullptr;
  double* d_ydiag = nullptr;  // |diag Z| per basis function (for diag_freq)
  double* d_sdiag = nullptr;  // diagonal of the Schur complement per node
  int diag_freq = -2;
  // aggregation multigrid preconditioner of the Schur complement CG (built for
  // amg_freq and amg_nr right-hand sides; device copies of every level)
  int schur_precond = 1;  // SVH_SCHUR_JACOBI / SVH_SCHUR_AMG
  int amg_freq = -2, amg_nr = 0;
  int amg_coarse = 0;  // kAmgCoarseDense / Diagonal / Jacobi
  struct AmgDev {
    int n = 0;
    int32_t *rptr = nullptr, *col = nullptr, *agg = nullptr, *mptr = nullptr, *mem = nullptr;
    double *val = nullptr, *dinv = nullptr;
    double2 *b = nullptr, *x = nullptr, *r = nullptr;  // [nr][n] work vectors
  };
  std::vector<AmgDev> amg;
  double* d_amg_cinv = nullptr;
  double schur_tol = 0;               // inner Schur CG relative tolerance (0: min(1e-8, rre))
  int verbose = -1;                   // solver progress on stderr (-1: read SVH_VERBOSE at the first solve)
  bool use_graphs = true;             // replay the captured PCG iteration block
  hipStream_t cap_stream = nullptr;   // private stream used only for graph capture
  // per-kernel timing: one event set per enqueued chunk while enabled
  bool prof = false;
  std::vector<std::vector<hipEvent_t>> prof_events;  // [tucker0, tucker1, x, y, z, yi, xi, end]
  std::vector<hipEvent_t> prof_pool;
  std::string err;
};

namespace svh {
// device launchers (return hipError_t)
hipError_t launch_even_spectrum(const svh_problem* p, const double* d_T, double* d_out,
                                double* d_tmp1, double* d_tmp2, hipStream_t s);
hipError_t launch_tucker_rebuild(const svh_problem* p, bool fp32_out, bool zspace, void* d_out,
                                 double* d_V, double* d_W, hipStream_t s);
// Tucker restoration of one family's z-space kernel rows (factor Fz3 has M3
// rows): out[m][ky][kx] = sum core F1 F2 Fz3.
hipError_t launch_tucker_rebuild_rows(const svh_problem* p, const DevTucker& t, const double* Fz3, int M3,
                                      bool fp32_out, void* d_out, double* d_V, double* d_W, hipStream_t s,
                                      bool xy_transposed = false);
// Restoration of a Tucker tensor on an n1 x n2 x n3 box (the factors' first
// n_i rows): out[k3][k2][k1]; scratch V (n1 d2 d3) and W (n1 n2 d3) doubles.
hipError_t launch_tucker_box(int n1, int n2, int n3, const DevTucker& t, const double* F3, bool fp32_out,
                             void* d_out, double* d_V, double* d_W, hipStream_t s);
// out[q][kx][ky] = in[dz_q][ky][kx] (z-space kernel rows of the fused path)
hipError_t launch_gather_transposed(const svh_problem* p, const double* d_in, double* d_out, hipStream_t s);
GeoT make_geo_t(const svh_problem* p, size_t csize);
int fused_phases(const svh_problem* p, size_t cs, size_t ts);
int yzy2_phases(const svh_problem* p);
bool fused_eligible(const svh_problem* p);
bool use_fused(const svh_problem* p, svh_prec prec);
// The first nfam (1 or 7) family tables [f][Kz][Ky][Kx] on the device by
// quadrature (M0, M1x, M1y, M1z, M2x, M2y, M2z).
hipError_t family_tables(const int K[3], int nfam, double* d_out, hipStream_t s);
// The first nfam tables for the problem's grid from the Toeplitz store (device).
hipError_t store_tables(const svh_problem* p, int nfam, double* d_out, hipStream_t s);
// z-space kernels of the seven families at the plane offsets dzset:
// rows [f][q][Ky][Kx] (device) -> out [f][q][Ly][Lx].
hipError_t launch_zspace_families(const svh_problem* p, const double* d_rows, int nd, double* d_out,
                                  double* d_tmp, hipStream_t s);
size_t tucker_scratch_doubles5(const svh_problem* p);
// Folded spectra (k_a <= L_a / 2) of nfam family tables; see tensors.hip.
hipError_t launch_folded_spectra(const svh_problem* p, const double* d_in, int nfam, double* d_out, double* d_tmp,
                                 hipStream_t s);
size_t folded_size(const svh_problem* p);
// Z step by zero-padded z FFT with the folded spectra (zfft.hip).
template <typename T>
hipError_t launch_zfft(const svh_problem* p, int nvec, void* B, const void* spec, hipStream_t s);
size_t zfft_lds_bytes(const svh_problem* p, size_t cs, int nc);
bool use_zdirect(const svh_problem* p);
Geo make_geo(const svh_problem* p, size_t csize);
void free_solver(svh_problem* p);
// y = Z x with element strides ldx, ldy between right-hand sides.
svh_status matvec_impl(svh_problem* p, svh_prec prec, int nrhs, const int32_t* freq_idx, const void* x,
                       long long ldx, void* y, long long ldy, void* ws, size_t ws_bytes, hipStream_t s);
size_t tucker_scratch_doubles(const svh_problem* p);
hipError_t launch_to_f32(const double* in, float* out, size_t n, hipStream_t s);

template <typename T>
hipError_t launch_matvec_chunk_fused(const svh_problem* p, int nvec, const EpiParams& ep, const void* x, void* y,
                                     void* A, void* O, const void* gk, hipStream_t s, hipEvent_t* ev);
template <typename T>
hipError_t launch_matvec_chunk(const svh_problem* p, int nvec, const EpiParams& ep,
                               const void* x, void* y, void* A, void* B, const void* zhat,
                               hipStream_t s, hipEvent_t* ev);
}  // namespace svh
