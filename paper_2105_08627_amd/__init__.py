"""Python binding of libsvh (the MI355X FFT-accelerated voxel VIE operator).

Argument marshalling only: every step of the operator runs in the HIP
library.  PyTorch supplies device memory and the current stream.  The
binding fails loudly when the library has not been built; there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsvh.so")

SVH_FP64, SVH_FP32, SVH_FP32_IR = 0, 1, 2
ZSTEP = {"auto": 0, "fft": 1, "direct": 2, "fused": 3}
_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENOTCONV", -5: "ESTATE"}

EXPORTED = [
    "svh_create", "svh_get_sizes", "svh_set_material", "svh_setup_tensors", "svh_green_toeplitz",
    "svh_get_toeplitz", "svh_get_family", "svh_set_green_method", "svh_toeplitz_store_build",
    "svh_set_toeplitz_store", "svh_toeplitz_store_restore", "svh_green_tables", "svh_tucker_compress", "svh_workspace_bytes", "svh_matvec", "svh_matvec_noalloc",
    "svh_set_zstep", "svh_autotune", "svh_set_ports", "svh_solve_sizes", "svh_solve_workspace_bytes", "svh_solve", "svh_set_graphs", "svh_set_schur_precond", "svh_set_schur_tol", "svh_matvec_adjoint", "svh_port_gradient", "svh_port_inductance", "svh_gradient_contract", "svh_profile_enable", "svh_profile_read", "svh_last_error", "svh_destroy",
]
PROF_NAMES = ["tucker_restore", "pass_x", "pass_y", "pass_z_mul", "pass_yi", "pass_xi"]

_lib = None


class SvhError(RuntimeError):
    pass


MAX_PORTS = 64


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("restarts", ctypes.c_int), ("inner_iterations", ctypes.c_int),
                ("refinement_steps", ctypes.c_int), ("converged", ctypes.c_int), ("relres", ctypes.c_double),
                ("relres_port", ctypes.c_double * MAX_PORTS)]


def lib():
    """Load libsvh.so (built in-tree by ``paper_2105_08627_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise SvhError(f"{LIB_PATH} is missing: build it with `python -m paper_2105_08627_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    L.svh_create.argtypes = [ctypes.POINTER(vp), i32, i32, i32, dbl, i32, vp]
    L.svh_get_sizes.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                ctypes.POINTER(i32)]
    L.svh_set_material.argtypes = [vp, i32, vp, vp, vp, i32]
    L.svh_setup_tensors.argtypes = [vp, vp]
    L.svh_green_toeplitz.argtypes = [i32, i32, i32, vp]
    L.svh_get_toeplitz.argtypes = [vp, vp]
    L.svh_get_family.argtypes = [vp, i32, vp]
    L.svh_set_green_method.argtypes = [vp, i32]
    L.svh_toeplitz_store_build.argtypes = [i32, i32, i32, i32, dbl, ctypes.c_char_p, vp, vp]
    L.svh_set_toeplitz_store.argtypes = [vp, ctypes.c_char_p]
    L.svh_toeplitz_store_restore.argtypes = [ctypes.c_char_p, i32, i32, i32, i32, vp, vp]
    L.svh_green_tables.argtypes = [i32, i32, i32, i32, vp, vp]
    L.svh_tucker_compress.argtypes = [vp, dbl, vp, vp]
    L.svh_workspace_bytes.argtypes = [vp, i32, i32]
    L.svh_workspace_bytes.restype = sz
    L.svh_matvec.argtypes = [vp, i32, i32, vp, vp, vp, vp, sz, vp]
    L.svh_matvec_noalloc.argtypes = [vp, i32, i32, vp, vp, vp, vp]
    L.svh_set_zstep.argtypes = [vp, i32]
    L.svh_set_ports.argtypes = [vp, i32, vp, vp, vp, vp]
    L.svh_set_graphs.argtypes = [vp, i32]
    L.svh_set_schur_precond.argtypes = [vp, i32]
    L.svh_set_schur_tol.argtypes = [vp, dbl]
    L.svh_matvec_adjoint.argtypes = [vp, i32, i32, vp, vp, vp, vp, sz, vp]
    L.svh_port_gradient.argtypes = [vp, i32, vp, vp, vp, vp]
    L.svh_port_inductance.argtypes = [vp, i32, vp, vp, vp]
    L.svh_gradient_contract.argtypes = [vp, i32, vp, vp, vp, vp, vp, sz, vp]
    L.svh_solve_sizes.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.svh_solve_workspace_bytes.argtypes = [vp, i32, i32]
    L.svh_solve_workspace_bytes.restype = sz
    L.svh_solve.argtypes = [vp, i32, i32, dbl, i32, i32, i32, vp, vp, ctypes.POINTER(SolveInfo), vp, sz, vp]
    L.svh_autotune.argtypes = [vp, i32, i32, vp, vp, vp, vp, sz, vp, vp]
    L.svh_profile_enable.argtypes = [vp, i32]
    L.svh_profile_read.argtypes = [vp, vp, vp]
    L.svh_last_error.argtypes = [vp]
    L.svh_last_error.restype = ctypes.c_char_p
    L.svh_destroy.argtypes = [vp]
    L.svh_destroy.restype = None
    for name in EXPORTED:
        if name not in ("svh_workspace_bytes", "svh_last_error", "svh_destroy", "svh_solve_workspace_bytes"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def green_toeplitz(Kx, Ky, Kz):
    """Host-only closed-form unit-voxel Green integral, array [Kz, Ky, Kx]."""
    T = np.zeros((Kz, Ky, Kx))
    st = lib().svh_green_toeplitz(Kx, Ky, Kz, _ptr(T))
    if st != 0:
        raise SvhError(f"svh_green_toeplitz: {_STATUS.get(st, st)}")
    return T


def toeplitz_store_build(K, nfam, tol, path, stream=None):
    """Algorithm 2, installation: Tucker-compressed unit-voxel tables of a
    K = (Kx, Ky, Kz) domain (nfam = 1 or 7 families) written to `path`.
    Returns the largest relative error bound of the families."""
    err = np.zeros(1)
    st = lib().svh_toeplitz_store_build(int(K[0]), int(K[1]), int(K[2]), int(nfam), float(tol),
                                        os.fsencode(path), _stream_handle(stream), _ptr(err))
    if st != 0:
        raise SvhError(f"svh_toeplitz_store_build: {_STATUS.get(st, st)}")
    return float(err[0])


def toeplitz_store_restore(path, K, nfam, out, stream=None):
    """Algorithm 2, execution: the first nfam tables for a K grid restored from
    the store into the device tensor `out` (float64, nfam * Kx * Ky * Kz)."""
    import torch
    _device_tensor(out, "out", torch.float64, min_numel=int(nfam) * int(K[0]) * int(K[1]) * int(K[2]))
    st = lib().svh_toeplitz_store_restore(os.fsencode(path), int(K[0]), int(K[1]), int(K[2]), int(nfam),
                                          ctypes.c_void_p(out.data_ptr()), _stream_handle(stream))
    if st != 0:
        raise SvhError(f"svh_toeplitz_store_restore: {_STATUS.get(st, st)}")
    return out


def green_tables(K, nfam, out, stream=None):
    """The first nfam unit-voxel tables computed on the device into `out`."""
    import torch
    _device_tensor(out, "out", torch.float64, min_numel=int(nfam) * int(K[0]) * int(K[1]) * int(K[2]))
    st = lib().svh_green_tables(int(K[0]), int(K[1]), int(K[2]), int(nfam), ctypes.c_void_p(out.data_ptr()),
                                _stream_handle(stream))
    if st != 0:
        raise SvhError(f"svh_green_tables: {_STATUS.get(st, st)}")
    return out


def _device_tensor(t, what, dtype, shape=None, min_numel=None):
    """Check a tensor handed to the library by pointer: the C calls take no
    shapes, so a wrong one would be read or written out of bounds."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(f"{what} holds {t.numel()} elements, {min_numel} needed")
    return t


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Problem:
    """One voxel grid with its material and circulant tensors (svh_problem)."""

    def __init__(self, mask, dx, basis=3):
        mask = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        if mask.ndim != 3:
            raise ValueError("mask must be [Kz, Ky, Kx]")
        self.Kz, self.Ky, self.Kx = mask.shape
        self.C = basis
        self._h = ctypes.c_void_p()
        st = lib().svh_create(ctypes.byref(self._h), self.Kx, self.Ky, self.Kz, float(dx), basis, _ptr(mask))
        if st != 0:
            raise SvhError(f"svh_create: {_STATUS.get(st, st)}")
        K, Lx, Ly, Lz = (ctypes.c_int() for _ in range(4))
        lib().svh_get_sizes(self._h, ctypes.byref(K), ctypes.byref(Lx), ctypes.byref(Ly), ctypes.byref(Lz))
        self.K = K.value
        self.L = (Lx.value, Ly.value, Lz.value)
        self._ws = {}

    def _check(self, st, what):
        if st != 0:
            msg = lib().svh_last_error(self._h).decode()
            raise SvhError(f"{what}: {_STATUS.get(st, st)}: {msg}")

    def set_material(self, freqs, sigma0, lam, per_voxel=False):
        f = np.ascontiguousarray(np.atleast_1d(np.asarray(freqs, dtype=np.float64)))
        s0 = np.ascontiguousarray(np.atleast_1d(np.asarray(sigma0, dtype=np.float64)))
        la = np.ascontiguousarray(np.atleast_1d(np.asarray(lam, dtype=np.float64)))
        self._check(lib().svh_set_material(self._h, f.size, _ptr(f), _ptr(s0), _ptr(la), int(per_voxel)),
                    "svh_set_material")

    def set_toeplitz_store(self, path):
        """Restore the tables from an Algorithm 2 store in later setup_tensors calls
        (None: compute them)."""
        self._check(lib().svh_set_toeplitz_store(self._h, None if path is None else os.fsencode(path)),
                    "svh_set_toeplitz_store")

    def set_green_method(self, method):
        """'quadrature' (device, default) or 'closed_form' (host binary128 M0)."""
        m = {"quadrature": 0, "closed_form": 1}[method]
        self._check(lib().svh_set_green_method(self._h, m), "svh_set_green_method")

    def setup_tensors(self, stream=None):
        self._check(lib().svh_setup_tensors(self._h, _stream_handle(stream)), "svh_setup_tensors")

    def toeplitz(self):
        T = np.zeros((self.Kz, self.Ky, self.Kx))
        self._check(lib().svh_get_toeplitz(self._h, _ptr(T)), "svh_get_toeplitz")
        return T

    def family(self, f):
        """Voxel-pair integral family f (0 M0, 1-3 M1x..M1z, 4-6 M2x..M2z), [Kz, Ky, Kx]."""
        T = np.zeros((self.Kz, self.Ky, self.Kx))
        self._check(lib().svh_get_family(self._h, int(f), _ptr(T)), "svh_get_family")
        return T

    def tucker_compress(self, tol):
        """Returns (ranks, relerr): ranks (d1, d2, d3) for basis 3, a 7 x 3
        array (one row per integral family) for basis 5."""
        nf = 7 if self.C == 5 else 1
        ranks = np.zeros(3 * nf, dtype=np.int32)
        err = np.zeros(1)
        self._check(lib().svh_tucker_compress(self._h, float(tol), _ptr(ranks), _ptr(err)), "svh_tucker_compress")
        self._ws.clear()
        if nf == 1:
            return tuple(int(r) for r in ranks), float(err[0])
        return ranks.reshape(nf, 3), float(err[0])

    def workspace_bytes(self, prec, nrhs):
        return int(lib().svh_workspace_bytes(self._h, prec, nrhs))

    def workspace(self, prec, nrhs, device):
        import torch
        key = (prec, nrhs)
        need = self.workspace_bytes(prec, nrhs)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint8, device=device)
            self._ws[key] = ws
        return ws

    def _batch(self, x, freq_idx, out):
        """Checks of a (nrhs, C, K) batch and its output; returns (prec, nrhs,
        freq_idx as int32, output tensor)."""
        import torch
        if not isinstance(x, torch.Tensor) or not x.is_cuda:
            raise ValueError("x must be a device tensor")
        if x.dtype == torch.complex128:
            prec = SVH_FP64
        elif x.dtype == torch.complex64:
            prec = SVH_FP32
        else:
            raise TypeError("x must be complex128 or complex64")
        if x.dim() != 3 or x.shape[0] < 1 or x.shape[1] != self.C or x.shape[2] != self.K:
            raise ValueError(f"x must have shape (nrhs, {self.C}, {self.K}), got {tuple(x.shape)}")
        _device_tensor(x, "x", x.dtype)
        nrhs = x.shape[0]
        fi = np.ascontiguousarray(np.broadcast_to(np.asarray(freq_idx, dtype=np.int32), (nrhs,)))
        if out is None:
            y = torch.empty_like(x)
        else:
            y = _device_tensor(out, "out", x.dtype, shape=x.shape)
            if y.device != x.device:
                raise ValueError("out must be on the device of x")
        return prec, nrhs, fi, y

    def matvec(self, x, freq_idx, out=None, stream=None):
        """y = Z x for x of shape (nrhs, C, K), complex128 (FP64) or complex64
        (FP32), on a CUDA device.  freq_idx: one slot per RHS (-1: bare)."""
        prec, nrhs, fi, y = self._batch(x, freq_idx, out)
        ws = self.workspace(prec, nrhs, x.device)
        st = lib().svh_matvec(self._h, prec, nrhs, _ptr(fi), ctypes.c_void_p(x.data_ptr()),
                              ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                              _stream_handle(stream))
        self._check(st, "svh_matvec")
        return y

    def matvec_noalloc(self, x, freq_idx, out, stream=None):
        """matvec with the library's static device workspace (svh_matvec_noalloc):
        no workspace tensor; `out` must be given (no output is allocated)."""
        prec, nrhs, fi, y = self._batch(x, freq_idx, out)
        st = lib().svh_matvec_noalloc(self._h, prec, nrhs, _ptr(fi), ctypes.c_void_p(x.data_ptr()),
                                      ctypes.c_void_p(y.data_ptr()), _stream_handle(stream))
        self._check(st, "svh_matvec_noalloc")
        return y

    def set_zstep(self, mode):
        """'auto', 'fft' (padded z FFT), 'direct' (z-space sum over occupied
        planes) or 'fused' (that sum with the y transforms in one kernel)."""
        self._check(lib().svh_set_zstep(self._h, ZSTEP[mode]), "svh_set_zstep")
        self._ws.clear()

    def autotune(self, x, freq_idx, stream=None):
        """Pick the fastest launch shapes for this batch; returns tuned ms/matvec."""
        prec, nrhs, fi, y = self._batch(x, freq_idx, None)
        ws = self.workspace(prec, nrhs, x.device)
        ms = np.zeros(1)
        self._check(lib().svh_autotune(self._h, prec, nrhs, _ptr(fi), ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                       _stream_handle(stream), _ptr(ms)), "svh_autotune")
        return float(ms[0])

    def set_ports(self, ports):
        """ports: list of (plus_faces, minus_faces); faces are (k, face code)
        pairs, face codes 0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z."""
        def csr(lists):
            ptr = np.zeros(len(lists) + 1, dtype=np.int32)
            flat = []
            for i, faces in enumerate(lists):
                flat.extend([int(v) for kf in faces for v in kf])
                ptr[i + 1] = ptr[i] + len(faces)
            return ptr, np.ascontiguousarray(np.asarray(flat, dtype=np.int32))
        pp, pf = csr([pl for pl, _ in ports])
        mp, mf = csr([mi for _, mi in ports])
        self._check(lib().svh_set_ports(self._h, len(ports), _ptr(pp), _ptr(pf), _ptr(mp), _ptr(mf)),
                    "svh_set_ports")
        N, M = ctypes.c_int(), ctypes.c_int()
        self._check(lib().svh_solve_sizes(self._h, ctypes.byref(N), ctypes.byref(M)), "svh_solve_sizes")
        self.N, self.M, self.nports = N.value, M.value, len(ports)

    def matvec_adjoint(self, x, freq_idx, out=None, stream=None):
        """y = Z^T x (same conventions as matvec)."""
        prec, nrhs, fi, y = self._batch(x, freq_idx, out)
        ws = self.workspace(prec, nrhs, x.device)
        self._check(lib().svh_matvec_adjoint(self._h, prec, nrhs, _ptr(fi), ctypes.c_void_p(x.data_ptr()),
                                             ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                             ws.numel(), _stream_handle(stream)), "svh_matvec_adjoint")
        return y

    def port_gradient(self, freq_idx, xfwd, xadj, stream=None):
        """dY[q, p, k] = d Y_qp / d (lambda_k^-2) from forward and adjoint solutions."""
        import torch
        if not hasattr(self, "nports"):
            raise SvhError("port_gradient: set_ports first")
        _device_tensor(xfwd, "xfwd", torch.complex128, shape=(self.nports, self.N))
        _device_tensor(xadj, "xadj", torch.complex128, shape=(self.nports, self.N))
        dY = torch.empty((self.nports, self.nports, self.K), dtype=torch.complex128, device=xfwd.device)
        self._check(lib().svh_port_gradient(self._h, int(freq_idx), ctypes.c_void_p(xfwd.data_ptr()),
                                            ctypes.c_void_p(xadj.data_ptr()), ctypes.c_void_p(dY.data_ptr()),
                                            _stream_handle(stream)), "svh_port_gradient")
        return dY

    def _admittance(self, Y):
        Yc = np.ascontiguousarray(np.asarray(Y, dtype=np.complex128))
        if Yc.shape != (self.nports, self.nports):
            raise ValueError(f"Y must be ({self.nports}, {self.nports})")
        return Yc

    def port_inductance(self, freq_idx, Y):
        """(Z, L): port impedance Y^-1 and inductance Im(Z)/w (svh_port_inductance)."""
        if not hasattr(self, "nports"):
            raise SvhError("port_inductance: set_ports first")
        Yc = self._admittance(Y)
        Z = np.zeros_like(Yc)
        L = np.zeros(Yc.shape)
        self._check(lib().svh_port_inductance(self._h, int(freq_idx), _ptr(Yc), _ptr(Z), _ptr(L)),
                    "svh_port_inductance")
        return Z, L

    def gradient_contract(self, freq_idx, Y, G, dY, stream=None):
        """grad[k] = sum_qp G[q,p] dL[q,p]/d(lambda_k^-2) (device float64 tensor),
        from the forward admittance Y, the loss weights G = dLoss/dL and dY of
        port_gradient (svh_gradient_contract)."""
        import torch
        if not hasattr(self, "nports"):
            raise SvhError("gradient_contract: set_ports first")
        _device_tensor(dY, "dY", torch.complex128, shape=(self.nports, self.nports, self.K))
        Yc = self._admittance(Y)
        Gc = np.ascontiguousarray(np.asarray(G, dtype=np.float64))
        if Gc.shape != (self.nports, self.nports):
            raise ValueError(f"G must be ({self.nports}, {self.nports})")
        g = torch.empty(self.K, dtype=torch.float64, device=dY.device)
        ws = torch.empty(16 * self.nports * self.nports, dtype=torch.uint8, device=dY.device)
        self._check(lib().svh_gradient_contract(self._h, int(freq_idx), _ptr(Yc), _ptr(Gc),
                                                ctypes.c_void_p(dY.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                                ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream)),
                    "svh_gradient_contract")
        return g

    def set_schur_precond(self, kind):
        """'amg' (default) or 'jacobi' preconditioning of the Schur-complement CG."""
        self._check(lib().svh_set_schur_precond(self._h, {"jacobi": 0, "amg": 1}[kind]), "svh_set_schur_precond")

    def set_schur_tol(self, tol):
        """Relative tolerance of the inner Schur-complement CG (0: the default)."""
        self._check(lib().svh_set_schur_tol(self._h, float(tol)), "svh_set_schur_tol")

    def set_graphs(self, enable):
        self._check(lib().svh_set_graphs(self._h, int(enable)), "svh_set_graphs")

    def solve(self, freq_idx, rre=1e-8, restart=50, maxit=1000, transpose=False, device="cuda", stream=None,
              check=True, refine=False):
        """Solve every port excitation; returns (X (nports, N) complex128 device
        tensor, Y admittance (nports, nports) numpy array, info dict)."""
        import torch
        X = torch.empty((self.nports, self.N), dtype=torch.complex128, device=device)
        prec = SVH_FP32_IR if refine else SVH_FP64
        nb = int(lib().svh_solve_workspace_bytes(self._h, prec, restart))
        ws = torch.empty(nb, dtype=torch.uint8, device=device)
        Y = np.zeros((self.nports, self.nports), dtype=np.complex128)
        info = SolveInfo()
        st = lib().svh_solve(self._h, prec, int(freq_idx), float(rre), int(restart), int(maxit),
                             int(transpose), ctypes.c_void_p(X.data_ptr()), _ptr(Y), ctypes.byref(info),
                             ctypes.c_void_p(ws.data_ptr()), nb, _stream_handle(stream))
        d = {"iterations": info.iterations, "restarts": info.restarts, "inner_iterations": info.inner_iterations,
             "refinement_steps": info.refinement_steps,
             "converged": bool(info.converged), "relres": info.relres,
             "relres_port": [info.relres_port[i] for i in range(self.nports)]}
        if st != 0 and not (st == -4 and not check):
            self._check(st, "svh_solve")
        return X, Y, d

    def profile(self, enable=True):
        self._check(lib().svh_profile_enable(self._h, int(enable)), "svh_profile_enable")

    def profile_read(self):
        """Per-kernel summed milliseconds since the last read, and call count."""
        ms = np.zeros(len(PROF_NAMES))
        n = np.zeros(1, dtype=np.int32)
        self._check(lib().svh_profile_read(self._h, _ptr(ms), _ptr(n)), "svh_profile_read")
        return dict(zip(PROF_NAMES, ms.tolist())), int(n[0])

    def close(self):
        if self._h:
            lib().svh_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
