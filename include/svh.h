/*
 * svh.h -- C ABI of the MI355X FFT-accelerated voxel VIE operator library.
 *
 * The library applies the Galerkin operator of the voxel volume integral
 * equation for superconducting structures (SuperVoxHenry, arXiv 2105.08627):
 * eq. 1 (VIE with the two-fluid conductivity of eq. 3), discretised with the
 * piecewise-constant basis of eq. 4 (three current components per voxel),
 * optionally with the two piecewise-linear functions of eqs. 5-6 (five per
 * voxel), whose block matrix (eq. 8) is applied through the FFT product of
 * eq. 9 with the circulant tensors rebuilt from their Tucker factors
 * (eqs. 10-11, Algorithm 1, Sec. II.B.2).
 *
 * Conventions used by every entry point
 *  - Voxels of the Kx x Ky x Kz grid are indexed x fastest, then y, then z.
 *    The K non-empty voxels (mask != 0) are numbered in that order.
 *  - Complex numbers are interleaved (re, im); FP64 entry points take
 *    double pairs, FP32 entry points float pairs.
 *  - A current vector holds C = 3 (basis 3) or C = 5 (basis 5) components,
 *    component-major: [I^x (K values); I^y (K); I^z (K); I^2D (K); I^3D (K)]
 *    (eq. 7).  A batch of nrhs vectors is stored back to back: element
 *    (rhs, comp, k) at (rhs*C + comp)*K + k.
 *  - Basis functions carry total current (f^x = x_hat / dx^2, and eqs. 5-6
 *    divided by dx^2), so that the voxel self terms are c/dx, c/(6 dx) and
 *    c/(2 dx) with c = 1/sigma (text under eq. 9, eqs. 16-18, 22-23) and the
 *    coupling is j*w*mu0*dx times unit-voxel Green integrals (App. B scaling
 *    with the basis normalisation); mu0 = 4*pi*1e-7 H/m.
 *  - Pointers named *_dev are device pointers (hipMalloc or torch CUDA
 *    tensors); *_host are host pointers read during the call only.  The
 *    library owns the problem object and its tensors; the caller owns every
 *    buffer it passes and must keep device buffers alive until the stream has
 *    passed the work enqueued on them.
 *  - Errors: every call returns an svh_status; on failure the problem's
 *    svh_last_error() text says why.  No call aborts the process.
 */
#ifndef SVH_H
#define SVH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SVH_OK = 0,
  SVH_EINVAL = -1,   /* bad argument (sizes, null pointers, ranges)            */
  SVH_ENOMEM = -2,   /* device or host allocation failed                       */
  SVH_EHIP = -3,     /* a HIP runtime call failed                               */
  SVH_ENOTCONV = -4, /* iterative method stopped before its tolerance           */
  SVH_ESTATE = -5    /* call made in the wrong order (e.g. matvec before setup) */
} svh_status;

/* SVH_FP32_IR (solve only): iterative refinement, FP64 residuals and
 * updates around inner solves whose operator runs in FP32. */
typedef enum { SVH_FP64 = 0, SVH_FP32 = 1, SVH_FP32_IR = 2 } svh_prec;

typedef struct svh_problem svh_problem;

/* Create a problem on the current HIP device.
 * Kx, Ky, Kz >= 1: voxel counts per axis (Sec. II.A: Kt = Kx*Ky*Kz).
 * dx_m > 0: voxel edge length in metres.
 * basis: 3 (piecewise-constant basis f^x, f^y, f^z of eq. 4) or 5 (plus the
 *   piecewise-linear f^2D, f^3D of eqs. 5-6, which let current turn corners).
 * mask_host: Kt bytes, x fastest; non-zero marks a non-empty voxel.  At least
 *   one voxel must be non-empty.
 * The FFT grid is L_i = 2 K_i when 2 K_i factors into 2s and 3s, else the
 * smallest such length >= 2 K_i - 1 (the circulant embedding of Sec. II.A
 * needs L_i >= 2 K_i - 1).  On success *out receives the new problem. */
svh_status svh_create(svh_problem** out, int Kx, int Ky, int Kz, double dx_m,
                      int basis, const uint8_t* mask_host);

/* Number of non-empty voxels K, and the FFT grid L (any pointer may be NULL). */
svh_status svh_get_sizes(const svh_problem* p, int* K, int* Lx, int* Ly, int* Lz);

/* Two-fluid material for nfreq frequencies (eq. 3; a, b of eqs. 22-23).
 * f_hz_host[nfreq] > 0; sigma0_host (S/m, >= 0) and lambda_host (London depth
 * in m, > 0) hold either one value each (per_voxel = 0) or K values each
 * (per_voxel = 1, compact voxel order).  Stores c = 1/sigma per frequency and
 * voxel on the device and the coupling scalar j*w*mu0*dx per frequency.
 * May be called again to replace the material. */
svh_status svh_set_material(svh_problem* p, int nfreq, const double* f_hz_host,
                            const double* sigma0_host, const double* lambda_host,
                            int per_voxel);

/* Toeplitz tensor of the unit-voxel Green integral (eq. 19 with the App. B
 * scaling, positive sign) for offsets [0,Kx) x [0,Ky) x [0,Kz) (with basis 5
 * also the M1/M2 families of eqs. 20-21), its circulant embedding (Sec. II.A)
 * and the spectrum of that circulant (the tensor Z of eq. 9 divided by
 * j*w*mu0*dx), or its z-space form, kept on the device in FP64.  The integrals
 * come from the method chosen with svh_set_green_method.
 * stream: a hipStream_t (NULL = default stream); the call returns after the
 * spectrum is complete. */
svh_status svh_setup_tensors(svh_problem* p, void* stream);

/* How svh_setup_tensors evaluates the voxel-pair integrals:
 *  SVH_GREEN_QUADRATURE  (default) all families on the device: tensor
 *                        Gauss-Legendre on the 8 polynomial boxes of the
 *                        overlap-weighted 3D form, point counts by distance
 *                        to the singular point; the 8 offsets whose boxes
 *                        touch it on the host, each box's monomial integrals
 *                        reduced exactly to regular face integrals (Euler's
 *                        relation for homogeneous functions and the
 *                        divergence theorem);
 *  SVH_GREEN_CLOSED_FORM M0 from the closed-form Coulomb box-box potential in
 *                        binary128 on the host (svh_green_toeplitz); the M1/M2
 *                        families still by quadrature.
 * The two agree to about 1e-15 of M0(0); the closed form is slower (seconds
 * for 8 M offsets on the host). */
#define SVH_GREEN_QUADRATURE 0
#define SVH_GREEN_CLOSED_FORM 1
svh_status svh_set_green_method(svh_problem* p, int method);

/* Toeplitz store (Algorithm 2, Sec. II.B.1).  Installation step: computes the
 * first nfam (1: M0; 7: all families of the linear basis) unit-voxel tables
 * for offsets [0,Kx) x [0,Ky) x [0,Kz) on the current device (quadrature),
 * Tucker-compresses each (Algorithm 1 on the Toeplitz tensor itself, relative
 * Frobenius tolerance tol), and writes the cores and factors to the file
 * `path` (overwritten).  relerr_out (may be NULL): largest bound-level error
 * estimate of the families.  Uses the device; returns when the file is
 * written. */
svh_status svh_toeplitz_store_build(int Kx, int Ky, int Kz, int nfam, double tol, const char* path,
                                    void* stream, double* relerr_out);

/* Algorithm 2, execution step on its own: restore the first nfam tables for
 * offsets [0,Kx) x [0,Ky) x [0,Kz) from the store file into T_dev (nfam*Kt
 * doubles, [f][z][y][x], device memory the caller owns).  EINVAL if the file
 * is unreadable, covers a smaller domain or holds fewer families.  Returns
 * when the tables are complete. */
svh_status svh_toeplitz_store_restore(const char* path, int Kx, int Ky, int Kz, int nfam, double* T_dev,
                                      void* stream);

/* The first nfam (1 or 7) unit-voxel tables computed directly (device
 * quadrature, as in svh_setup_tensors) into T_dev (nfam*Kt doubles, device).
 * Returns when they are complete. */
svh_status svh_green_tables(int Kx, int Ky, int Kz, int nfam, double* T_dev, void* stream);

/* Use the store file `path` in later svh_setup_tensors calls of p: the tables
 * of p's grid are restored from the factors' leading rows (the trim of
 * Algorithm 2) on the device instead of being computed.  The stored domain
 * must cover the grid, and basis 5 needs a seven-family store (EINVAL
 * otherwise).  The factors are read now and kept in host memory; path = NULL
 * stops using a store.  (The (dx)^5 scale of Algorithm 2 is part of the
 * coupling j*w*mu0*dx applied per frequency.) */
svh_status svh_set_toeplitz_store(svh_problem* p, const char* path);

/* Host-only: the unit-voxel Green integral of eq. 19 (positive sign, App. B
 * with dx = 1) for offsets [0,Kx) x [0,Ky) x [0,Kz), written to T_host
 * (Kt doubles, offsets x fastest).  Evaluated from the closed-form Coulomb
 * box-box potential in binary128 arithmetic.  Touches no GPU. */
svh_status svh_green_toeplitz(int Kx, int Ky, int Kz, double* T_host);

/* Copy the Toeplitz tensor computed by svh_setup_tensors to the host
 * (Kt doubles, offsets x fastest). */
svh_status svh_get_toeplitz(const svh_problem* p, double* T_host);

/* Copy one voxel-pair integral family computed by svh_setup_tensors (Kt
 * doubles for offsets [0,Kx) x [0,Ky) x [0,Kz), x fastest; unit voxels,
 * positive sign).  For source point u' and observer point u measured from
 * their voxel centres and g = 1/(4 pi |r|) (eq. 8, App. A eqs. 19-21):
 *   family 0  M0   = int int g
 *   family 1-3  M1_a = int int u'_a g   (a = x, y, z; odd along a)
 *   family 4-6  M2_a = int int u_a u'_a g
 * Family 0 is the closed form of svh_green_toeplitz; families 1-6 (basis 5
 * only, EINVAL otherwise) are computed by Gauss-Legendre quadrature of the
 * overlap-weighted 3D form on the device (the offsets whose boxes touch the
 * singular point on the host, reduced to regular face integrals). */
svh_status svh_get_family(const svh_problem* p, int family, double* T_host);

/* Tucker-compress the circulant spectrum (Algorithm 1, Sec. II.B.2) with
 * relative Frobenius tolerance tol >= 0 (tol/sqrt(3) per mode).  After this
 * call every matvec restores the spectrum from the Tucker factors (eq. 10)
 * instead of keeping it resident, and the dense spectrum is freed.
 * Basis 5 compresses the spectrum of each of the seven integral families
 * separately (each to its own relative tolerance).
 * ranks_out (may be NULL): multilinear ranks d1, d2, d3 per family (3 ints
 *   for basis 3, 7 x 3 ints for basis 5 in family order).
 * relerr_out (may be NULL): bound-level estimate sqrt(sum of discarded
 * squared singular values) / ||Z||_F summed over the three modes (largest
 * over the families). */
svh_status svh_tucker_compress(svh_problem* p, double tol, int32_t* ranks_out,
                               double* relerr_out);

/* Bytes of device workspace svh_matvec needs for nrhs right-hand sides. */
size_t svh_workspace_bytes(const svh_problem* p, svh_prec prec, int nrhs);

/* y = Z x for nrhs right-hand sides (eq. 9 plus the diagonal z^beta I^beta).
 * prec: SVH_FP64 (x, y complex double) or SVH_FP32 (complex float; the
 *   Tucker restoration still accumulates in FP64 and is rounded once).
 * freq_idx_host[nrhs]: frequency slot (from svh_set_material) per RHS, or -1
 *   for the bare unit-voxel convolution y = T * x (no j*w*mu0*dx factor and
 *   no diagonal term).
 * x_dev, y_dev: nrhs*C*K complex values each (layout above); must not
 *   overlap.  ws_dev: at least svh_workspace_bytes(p, prec, nrhs) bytes.
 * stream: hipStream_t on which all work is enqueued; the call does not
 *   synchronise. */
svh_status svh_matvec(svh_problem* p, svh_prec prec, int nrhs,
                      const int32_t* freq_idx_host, const void* x_dev, void* y_dev,
                      void* ws_dev, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as svh_matvec, with the workspace taken from a fixed array of
 * 64 MiB in device memory (one per device, reserved when the library's code
 * is loaded on that device and held until the process ends) instead of a
 * caller buffer.  Makes no allocation (no hipMalloc, no events).  The
 * caller still passes x_dev and y_dev (as in svh_matvec).
 * EINVAL if svh_workspace_bytes(p, prec, nrhs) exceeds 64 MiB (the text of
 * svh_last_error gives the size needed; call svh_matvec with a workspace
 * then), or if the current device is not the one p was created on;
 * ESTATE while per-kernel profiling is enabled.  Every call on one device
 * shares that array: calls that may overlap on one device (several streams
 * or threads) race and give wrong results; serialise them.  Nothing in the
 * array needs to start at zero (every byte the product reads it first
 * writes in the same call).  Enqueued on stream; does not synchronise. */
svh_status svh_matvec_noalloc(svh_problem* p, svh_prec prec, int nrhs, const int32_t* freq_idx_host,
                              const void* x_dev, void* y_dev, void* stream);

/* Autotuner: times the launch shapes of the FFT passes (persistent grids of
 * 1, 2 or 4 resident waves of blocks, or one block per pencil group; full or
 * half column tiles for the y passes) on this exact batch (same arguments as
 * svh_matvec), keeps the fastest shape per pass for later svh_matvec calls in
 * precision prec, in SVH_ZSTEP_AUTO mode also times the fused step against the
 * separate passes and keeps the faster, and synchronises the stream.  y_dev
 * is overwritten.  ms_out (may be NULL): kernel time of one tuned matvec in
 * milliseconds. */
svh_status svh_autotune(svh_problem* p, svh_prec prec, int nrhs, const int32_t* freq_idx_host,
                        const void* x_dev, void* y_dev, void* ws_dev, size_t ws_bytes, void* stream,
                        double* ms_out);

/* Per-kernel timing of svh_matvec with HIP events recorded on the call's
 * stream (for measurement; off by default).  While enabled every matvec
 * records events around each kernel. */
#define SVH_NPROF 6
svh_status svh_profile_enable(svh_problem* p, int enable);

/* Sum, over the matvec calls since the last read, of the kernel durations in
 * milliseconds: ms_out[SVH_NPROF] = {Tucker restoration, X pass, Y pass,
 * Z pass (forward z FFT, spectrum product, inverse z FFT), inverse Y pass,
 * inverse X pass with the diagonal term}.  ncalls_out (may be NULL) receives
 * the number of kernel sequences summed.  Waits for the recorded events. */
svh_status svh_profile_read(svh_problem* p, double* ms_out, int* ncalls_out);

/* Choice of the z-direction step of the product (all choices give the same
 * operator up to rounding):
 *  SVH_ZSTEP_AUTO   (default) DIRECT when at most 32 planes are occupied
 *                   (basis 5: and at most 64 distinct plane offsets), else
 *                   FFT; svh_autotune switches a precision to FUSED
 *                   when that applies (basis 3, at most 32 occupied z planes
 *                   with at most 64 distinct plane offsets) and it timed the
 *                   fused step faster on the caller's batch;
 *  SVH_ZSTEP_FFT    zero-padded FFT along z, product with the circulant
 *                   spectrum (basis 5: the 17 blocks of eq. 8 from the seven
 *                   family spectra), inverse FFT (eq. 9 literally);
 *  SVH_ZSTEP_DIRECT after the x and y transforms, the Toeplitz sum along z
 *                   over the occupied planes with the inverse z transform of
 *                   the circulant spectrum (EINVAL if more than 32 planes);
 *  SVH_ZSTEP_FUSED  the same sum, with the y transform, the z sum and the
 *                   inverse y transform of one x frequency in one kernel
 *                   (EINVAL where it does not apply).
 * FUSED applies to basis 3 only. */
#define SVH_ZSTEP_AUTO 0
#define SVH_ZSTEP_FFT 1
#define SVH_ZSTEP_DIRECT 2
#define SVH_ZSTEP_FUSED 3
svh_status svh_set_zstep(svh_problem* p, int mode);

/* ---------------------------------------------------------------- solve --
 * Saddle system of eq. 7 with ports.  Nodes are the centres of the faces of
 * non-empty voxels; A[m, (k, a)] is the current basis f^a of voxel k draws
 * from node m (+1 at its -a face, -1 at its +a face), so A I = 0 is current
 * conservation (eq. 2) and the first block row reads Z I - A^T Phi = V.
 * The linear functions draw -1/2 through both x faces and +1/2 through both
 * y faces (f^2D), -1/2 through the four x and y faces and +1 through both z
 * faces (f^3D).
 * A port holds Phi = 1 on its + terminal faces and Phi = 0 on its - terminal
 * faces and on the faces of every other port.  Each conductor region without
 * a port face has one node grounded (its potential is otherwise undefined).
 * The admittance Y[q][p] is the current entering port q's + terminal when
 * port p is driven (b_q^T I_p with b_q = A_{q+}^T 1); Y^-1 is the port
 * impedance matrix and Im(Y^-1)/w the inductance matrix. */
#define SVH_MAX_PORTS 64

/* Define the ports.  Faces are (voxel index k in compact order, face code)
 * pairs with face codes 0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z.  Port q's +
 * terminal faces are plus_faces[2*i .. 2*i+1] for plus_ptr[q] <= i <
 * plus_ptr[q+1] (minus likewise); 1 <= nports <= SVH_MAX_PORTS.  Builds the
 * node topology on first use.  Host arrays, read during the call. */
svh_status svh_set_ports(svh_problem* p, int nports, const int32_t* plus_ptr, const int32_t* plus_faces,
                         const int32_t* minus_ptr, const int32_t* minus_faces);

/* Preconditioner of the conjugate-gradient solve of the Schur complement
 * S = A_F Y^-1 A_F^T inside the preconditioner of eqs. 12-15:
 *  SVH_SCHUR_JACOBI  diagonal of S;
 *  SVH_SCHUR_AMG     (default) one symmetric V-cycle of an aggregation
 *                    multigrid (pairwise aggregation, aggregates of up to four
 *                    nodes, Galerkin coarse matrices, damped Jacobi smoothing,
 *                    exact coarsest solve), built on the host at the first
 *                    solve of a frequency.
 * Both give the same solution to the solve tolerance. */
#define SVH_SCHUR_JACOBI 0
#define SVH_SCHUR_AMG 1
svh_status svh_set_schur_precond(svh_problem* p, int kind);

/* Relative residual tolerance of the conjugate-gradient solve of the Schur
 * complement inside the preconditioner (eqs. 13-15).  The outer method is
 * flexible GMRES, which admits an inexact preconditioner, so a loose inner
 * tolerance trades inner steps for outer ones.  0 (default): rre clamped to
 * [1e-12, 1e-8] in FP64 solves; 1e-4 in the refinement's inner solves, whose
 * conjugate gradients run in FP32.  EINVAL unless 0 <= tol < 1.  Setting
 * SVH_VERBOSE=1 in the environment makes svh_solve print one progress line
 * per GMRES cycle and refinement step on stderr. */
svh_status svh_set_schur_tol(svh_problem* p, double tol);

/* Unknowns per port column N = C K + M and node count M (after svh_set_ports). */
svh_status svh_solve_sizes(const svh_problem* p, int* N, int* M);

typedef struct {
  int iterations;        /* outer (F)GMRES steps                              */
  int restarts;          /* restart cycles                                     */
  int inner_iterations;  /* conjugate-gradient steps in the preconditioner    */
  int refinement_steps;  /* outer refinement steps (SVH_FP32_IR)              */
  int converged;         /* 1 if every port reached the tolerance             */
  double relres;         /* largest true relative residual ||b - K x|| / ||b|| */
  double relres_port[SVH_MAX_PORTS];
} svh_solve_info;

/* Workspace bytes of svh_solve for restart length `restart`. */
size_t svh_solve_workspace_bytes(const svh_problem* p, svh_prec prec, int restart);

/* Solve K x_p = [b_p; 0] for every port p (right-preconditioned flexible
 * GMRES with restart `restart`, Sec. III; the preconditioner is eq. 12 with
 * Y = |diag Z| applied through eqs. 13-15, its Schur complement solved by
 * conjugate gradients to a relative 1e-8 or rre, whichever is smaller).
 * prec: SVH_FP64, or SVH_FP32_IR: refinement steps x += d with the residual
 *   b - K x formed in FP64 and d from one cycle of an inner flexible GMRES
 *   (relative tolerance max(1e-6, rre)) whose Z products and Schur-complement
 *   conjugate gradients run in FP32 (Tucker restoration accumulation, Krylov
 *   vectors and orthogonalisation stay FP64).  The Arnoldi steps run without
 *   host synchronisation (Hessenberg columns, Givens rotations and back
 *   substitution on the device) and are replayed from captured HIP graphs
 *   (svh_set_graphs).  freq_idx: frequency slot of the material.  rre: relative
 * residual target (the paper uses 1e-8).  maxit: cap on GMRES steps.
 * transpose != 0 solves K^T x = [b; 0] instead (adjoint system).
 * x_dev: nports columns of N complex doubles (currents, component-major as in
 * svh_matvec, then node potentials; port and grounded nodes hold 0).  Nodes
 * are numbered in face-grid order: faces normal to x, then y, then z, each
 * set with x fastest, then y, then z, counting only faces of non-empty
 * voxels.
 * Y_host (may be NULL): nports*nports complex doubles, Y[q*nports + p].
 * info (may be NULL): iteration counts and true residuals.
 * Returns SVH_ENOTCONV (with x, Y and info filled) if the target is missed.
 * Synchronises the stream. */
svh_status svh_solve(svh_problem* p, svh_prec prec, int freq_idx, double rre, int restart, int maxit,
                     int transpose, void* x_dev, double* Y_host, svh_solve_info* info, void* ws_dev,
                     size_t ws_bytes, void* stream);

/* Replay each Arnoldi step of svh_solve (preconditioner with its fixed
 * number of conjugate-gradient steps, operator, Gram-Schmidt, Givens) from a
 * HIP graph captured once per Krylov column and solve (default 1), or launch
 * the same kernels one by one (0); both give bitwise the same result. */
svh_status svh_set_graphs(svh_problem* p, int enable);

/* y = Z^T x (transpose, not conjugate transpose), same arguments and layout
 * as svh_matvec.  Used by the adjoint solve (svh_solve with transpose = 1)
 * and the gradient below. */
svh_status svh_matvec_adjoint(svh_problem* p, svh_prec prec, int nrhs, const int32_t* freq_idx_host,
                              const void* x_dev, void* y_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* Gradient of the port admittance with respect to the per-voxel kinetic
 * parameter p_k = lambda_k^-2 (eq. 3).  xfwd_dev: forward solutions of
 * svh_solve (transpose = 0); xadj_dev: adjoint solutions (transpose = 1),
 * both nports columns of N complex doubles, at the same frequency slot and
 * material.  dY_dev receives nports*nports*K complex doubles,
 * dY[(q*nports + p)*K + k] = d Y[q][p] / d p_k.  Enqueued on stream. */
svh_status svh_port_gradient(svh_problem* p, int freq_idx, const void* xfwd_dev, const void* xadj_dev,
                             void* dY_dev, void* stream);

/* Port impedance and inductance from the admittance of svh_solve (eq. 3 and
 * the inductance extraction of Sec. III): Z = Y^-1 and L = Im(Z) / w, with w
 * the angular frequency of slot freq_idx.  Y_host: nports*nports complex
 * doubles, Y[q*nports + p] (as svh_solve writes it).  Z_host (may be NULL):
 * nports*nports complex doubles; L_host (may be NULL): nports*nports doubles
 * in henry.  Host arithmetic only (Gauss-Jordan elimination with partial
 * pivoting); EINVAL if Y is singular.  Touches no GPU. */
svh_status svh_port_inductance(svh_problem* p, int freq_idx, const double* Y_host, double* Z_host,
                               double* L_host);

/* Gradient of a scalar loss of the port inductances with respect to the
 * per-voxel kinetic parameter p_k = lambda_k^-2 (eq. 3):
 *   grad_dev[k] = sum_{q,p} G[q][p] dL[q][p] / dp_k,  L = Im(Y^-1) / w,
 * computed as -(1/w) Im( sum_{a,b} W[a][b] dY[a][b][k] ) with W = Z^T G Z^T,
 * Z = Y^-1 (dZ = -Z dY Z).  Y_host: the admittance of the forward solve
 * (nports^2 complex doubles); G_host: dLoss/dL, nports^2 doubles, row-major
 * [q][p]; dY_dev from svh_port_gradient at the same frequency slot; grad_dev:
 * K doubles (device).  ws_dev: device workspace of at least 16*nports^2
 * bytes (receives W).  EINVAL if Y is singular.  Synchronises the stream. */
svh_status svh_gradient_contract(svh_problem* p, int freq_idx, const double* Y_host, const double* G_host,
                                 const void* dY_dev, double* grad_dev, void* ws_dev, size_t ws_bytes,
                                 void* stream);

/* Text of the last error on this problem (never NULL). */
const char* svh_last_error(const svh_problem* p);

/* Release the problem and all library-owned device memory. */
void svh_destroy(svh_problem* p);

#ifdef __cplusplus
}
#endif

#endif /* SVH_H */
