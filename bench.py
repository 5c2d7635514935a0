"""Benchmark of the batched FFT-VIE matrix-vector product on one MI355X.

One step = one batched application of the operator (Tucker restoration of the
circulant spectrum, then the five FFT / product passes and the diagonal term)
to every right-hand side of the workload: the 256 x 256 x 128 three-layer
stack, 8 ports x 8 frequencies = 64 right-hand sides, three current
components each.  Inputs are resident in HBM before the timed region.

Prints one JSON line (metric, value = FP32 matvecs/s, FP64 figures beside it,
roofline of the dominant kernel, oracle CPU baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# device kernel of each timed step on the stack workload, FP32
KERNEL_NAMES_FP32 = {
    "pass_x": "svh::k_pass_x<float, svh::PlanC<8, 8, 8, 1> >",
    "pass_y": "svh::k_pass_y<float, -1, svh::PlanC<8, 8, 8, 1> >",
    "pass_z_mul": "svh::k_zdirect<float, 24, 8, 4, 512>",
    "pass_yi": "svh::k_pass_y<float, 1, svh::PlanC<8, 8, 8, 1> >",
    "pass_xi": "svh::k_pass_xi<float, svh::PlanC<8, 8, 8, 1> >",
}
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
# the library is built without packed FP32 instructions: one FP32 FMA per lane
# per clock, 256 CUs x 64 lanes x 2 FLOP x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 78.6


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    """sha256 of the library's kernel sources (csrc/*, sorted by name)."""
    import hashlib
    d = os.path.join(ROOT, "paper_2105_08627_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".h", ".cpp")):
            h.update(name.encode())
            with open(os.path.join(d, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel_name):
    """HBM bytes per launch of `kernel_name` from the committed counter summary
    (rocprofv3 FETCH_SIZE and WRITE_SIZE per dispatch, scaled by the factors a
    plain device copy of known size gives), or None when the summary was taken
    from other kernel sources than the ones built now."""
    path = os.path.join(ROOT, "profiles", "counters_c5_stack.txt")
    if not os.path.exists(path):
        return None
    rows, meta = {}, {}
    with open(path) as f:
        for line in f:
            parts = line.split("\t")
            if len(parts) == 2:
                meta[parts[0].strip()] = parts[1].strip()
            elif len(parts) == 3 and parts[0] != "kernel":
                rows[parts[0].strip()] = (float(parts[1]), float(parts[2]))
    if meta.get("source_sha256") != kernel_source_hash() or kernel_name not in rows:
        return None
    fk, wk = rows[kernel_name]
    return 1024.0 * (fk * float(meta["fetch_factor"]) + wk * float(meta["write_factor"]))


def pass_bytes(p, nvec, cs, ts, K, nzp, nd):
    """Algorithmic HBM bytes of each kernel for one launch over nvec vectors.

    X  : read compact x, write the x-transformed planes (nzp * Ky * Lx)
    Y  : read those, write nzp * Ly * Lx
    Z  : read and write nzp * Ly * Lx, read the kernel once: the z-space
         kernel at the nd distinct plane offsets (direct z step), else the
         spectrum (Lx Ly Lz)
    Yi : read nzp * Ly * Lx, write nzp * Ky * Lx
    Xi : read nzp * Ky * Lx and compact x and c/dx, write compact y
    """
    Lx, Ly, Lz = p.L
    Ky = p.Ky
    a = nzp * Ky * Lx * cs
    b = nzp * Ly * Lx * cs
    v = K * cs
    return {
        "pass_x": nvec * (v + a),
        "pass_y": nvec * (a + b),
        "pass_z_mul": nvec * 2 * b + Lx * Ly * (nd if nzp <= 32 else Lz) * ts,
        "pass_yi": nvec * (b + a),
        "pass_xi": nvec * (a + 3 * v),
    }


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_worker(workload, nrhs, sample_rows, budget_s):
    """Child process of the CPU baselines (started before the GPU is touched;
    stdin/stdout carry the handshake).  Builds the oracle's M0 table for the
    grid (untimed, while the GPU sections run), prints READY, waits for GO on
    stdin, then times
      * the oracle's dense row sum (``operator.dense_rows`` and the product
        with the right-hand sides, as ``operator.dense_matvec`` does) on a
        seeded sample of observer rows, extrapolated to full products;
      * a plain FP64 FFT product (eq. 9 with the same circulant embedding,
        ``scipy.fft`` on every host core) for one right-hand side,
    and prints one JSON line with both."""
    import scipy.fft as sfft
    import workloads as wl
    from oracle import operator as op
    cfg = wl.WORKLOADS[workload]
    mask = cfg["mask"]()
    Kz, Ky, Kx = mask.shape
    dx, freqs, sigma0, lam = cfg["dx"], cfg["freqs"], cfg["sigma0"], cfg["lam"]
    nf = len(freqs)
    fidx = [r % nf for r in range(nrhs)]
    x = wl.random_currents(cfg["seed"], (nrhs, 3, int(mask.sum())))
    P = op.voxel_coords(mask)
    K = P.shape[0]
    fam = op.FamilyCache(Kx, Ky, Kz)
    t = time.perf_counter()
    fam.table("M0")
    t_table = time.perf_counter() - t
    L = [2 * k for k in (Kx, Ky, Kz)]
    t = time.perf_counter()
    H = sfft.fftn(op.embed(lambda o: fam.values("M0", o), (Kx, Ky, Kz), L), workers=-1).real
    t_spec = time.perf_counter() - t
    print("READY", flush=True)
    sys.stdin.readline()
    cores = len(os.sched_getaffinity(0))
    # dense row sum: rows (beta, l) for every right-hand side, grouped by frequency
    rng = np.random.default_rng(7)
    rows = rng.choice(3 * K, size=sample_rows, replace=False)
    X = x.reshape(nrhs, 3 * K)
    done = 0
    t0 = time.perf_counter()
    while done < len(rows) and time.perf_counter() - t0 < budget_s:
        row = rows[done:done + 1]
        for f in range(nf):
            sel = [r for r in range(nrhs) if fidx[r] == f]
            s = 1j * 2 * np.pi * freqs[f] * op.MU0 * dx
            c = op.material_c(freqs[f], sigma0, lam) * np.ones(K)
            Zr = op.dense_rows(mask, 3, row, fam, s, c, dx)
            _ = X[sel] @ Zr.T
        done += 1
    dt = time.perf_counter() - t0
    dense = {"value": nrhs * done / (3 * K) / dt, "unit": "matvecs/s", "cores": cores, "kind": "oracle",
             "sample": f"{done} of the {3 * K} operator rows (each for all {nrhs} RHS at their {nf} frequencies) "
                       f"of the oracle's dense O(N^2) row sum, {dt:.1f} s, extrapolated to whole products; "
                       f"the M0 table ({Kx}x{Ky}x{Kz} offsets, {t_table:.0f} s) built before timing",
             "cpu_model": cpu_model()}
    # FFT product, FP64, one right-hand side (three components)
    s = 1j * 2 * np.pi * freqs[fidx[0]] * op.MU0 * dx
    c = op.material_c(freqs[fidx[0]], sigma0, lam)
    nrep = 0
    t0 = time.perf_counter()
    while nrep < 2:
        y = np.empty((3, K), dtype=np.complex128)
        for a in range(3):
            g = np.zeros((L[2], L[1], L[0]), dtype=np.complex128)
            g[P[:, 2], P[:, 1], P[:, 0]] = x[0, a]
            G = sfft.fftn(g, workers=-1)
            G *= H
            y[a] = s * sfft.ifftn(G, workers=-1)[P[:, 2], P[:, 1], P[:, 0]] + c / dx * x[0, a]
        nrep += 1
    dt_fft = time.perf_counter() - t0
    fftb = {"value": nrep / dt_fft, "unit": "matvecs/s", "cores": cores, "kind": "scipy.fft FP64",
            "sample": f"{nrep} products of one RHS (3 components): zero-pad to {L[0]}x{L[1]}x{L[2]}, "
                      f"3 forward and 3 inverse FFTs, spectrum product, crop, diagonal; scipy.fft workers = all "
                      f"{cores} cores; spectrum built before timing ({t_spec:.0f} s)",
            "cpu_model": cpu_model()}
    print(json.dumps({"dense": dense, "fft": fftb}), flush=True)


class CpuBaseline:
    """Runs cpu_worker in a child process started before the GPU is used."""

    def __init__(self, workload, nrhs, sample_rows=2048, budget_s=20.0):
        import subprocess
        self.p = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", workload,
                                   "--nrhs", str(nrhs), "--cpu-rows", str(sample_rows),
                                   "--cpu-budget", str(budget_s)],
                                  stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True)

    def result(self):
        line = self.p.stdout.readline()
        if not line.startswith("READY"):
            self.p.kill()
            raise RuntimeError(f"cpu baseline worker failed: {line!r}")
        self.p.stdin.write("GO\n")
        self.p.stdin.flush()
        out = self.p.stdout.readline()
        self.p.wait()
        return json.loads(out)


def bench_basis5(args, cfg, mask, fidx, dev):
    """The same workload with the piecewise-linear basis (five components per
    voxel, eqs. 5-6): seven integral families, each Tucker-compressed to the
    same tolerance, coupled five-component z step."""
    import torch
    import paper_2105_08627_amd as svh
    import workloads as wl
    dx, freqs, sigma0, lam = cfg["dx"], cfg["freqs"], cfg["sigma0"], cfg["lam"]
    nrhs = len(fidx)
    t = time.perf_counter()
    p = svh.Problem(mask, dx, basis=5)
    p.set_material(freqs, sigma0, lam)
    p.setup_tensors()
    if args.zstep in ("auto", "fft", "direct"):
        p.set_zstep(args.zstep)
    t_setup = time.perf_counter() - t
    t = time.perf_counter()
    ranks, terr = p.tucker_compress(args.tol)
    t_tucker = time.perf_counter() - t
    log(f"[bench] basis5 setup {t_setup:.1f}s tucker {t_tucker:.1f}s ranks {ranks.tolist()} bound {terr:.2e}")
    K = p.K
    nzp = int(np.count_nonzero(mask.reshape(mask.shape[0], -1).any(axis=1)))
    x64 = torch.from_numpy(wl.random_currents(cfg["seed"] + 5, (nrhs, 5, K))).to(dev)
    x32 = x64.to(torch.complex64)
    y32, y64 = torch.empty_like(x32), torch.empty_like(x64)
    p.autotune(x32, fidx)
    p.autotune(x64, fidx)
    res = {}
    for name, x, y, steps in (("fp32", x32, y32, max(args.steps // 2, 1)), ("fp64", x64, y64, args.fp64_steps)):
        p.matvec(x, fidx, out=y)
        torch.cuda.synchronize()
        p.profile(True)
        p.profile_read()
        t0 = time.perf_counter()
        for _ in range(steps):
            p.matvec(x, fidx, out=y)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof, ncall = p.profile_read()
        p.profile(False)
        per = {k: v / steps for k, v in prof.items()}  # one profile set per launch chunk
        res[name] = {"value": nrhs * steps / dt, "unit": "matvecs/s", "ms_per_step": dt * 1e3 / steps,
                     "kernels_ms_per_step": per}
        log(f"[bench] basis5 {name} {steps} steps {dt * 1e3 / steps:.3f} ms/step  "
            + " ".join(f"{k}={v:.3f}" for k, v in per.items()))
    rel = (torch.linalg.vector_norm((y32.to(torch.complex128) - y64).flatten())
           / torch.linalg.vector_norm(y64.flatten())).item()

    # adjoint product (same kernels through the transposed block table)
    ya32, adj32 = bench_adjoint(p, x32, fidx, max(args.steps // 2, 1))
    ya64, adj64 = bench_adjoint(p, x64, fidx, args.fp64_steps)
    adj_sym = (torch.linalg.vector_norm((ya64 - y64).flatten()) / torch.linalg.vector_norm(y64.flatten())).item()
    del ya32, ya64
    log(f"[bench] basis5 adjoint fp32 {adj32['ms_per_step']:.3f} ms/step fp64 {adj64['ms_per_step']:.3f} ms/step "
        f"|Z^T x - Z x|/|Z x| {adj_sym:.1e}")
    Lx, Ly, _ = p.L
    # coupled z step: 12 z convolutions of complex data with real kernels per
    # pencil, i.e. 48 flops per (pencil, RHS, observer plane, source plane);
    # on the matrix cores (FP32, up to 24 planes) the observer planes are
    # padded to 16-row tiles and the source planes to the 8/16/24 bucket
    zflops = 48.0 * nrhs * Lx * Ly * nzp * nzp
    nzb = 8 if nzp <= 8 else 16 if nzp <= 16 else 24
    zflops_mfma = 48.0 * nrhs * Lx * Ly * (16 * ((nzb + 15) // 16)) * nzb if nzp <= 24 else None
    zms = res["fp32"]["kernels_ms_per_step"]["pass_z_mul"]
    zs = np.nonzero(mask.reshape(mask.shape[0], -1).any(axis=1))[0]
    nd = len({abs(int(a) - int(b)) for a in zs for b in zs})
    by = pass_bytes(p, 5 * nrhs, 8, 4, K, nzp, nd)
    by["pass_z_mul"] = 5 * nrhs * 2 * nzp * Ly * Lx * 8 + 7 * nd * Lx * Ly * 4
    return {"workload": f"same grid and RHS, piecewise-linear basis: 5 components, K={K}, "
                        f"7 integral families, Tucker tol {args.tol:g}",
            "setup_s": t_setup, "tucker_s": t_tucker, "tucker_ranks": ranks.tolist(),
            **res, "rel_err_fp32_vs_fp64": rel,
            "adjoint": {"fp32": adj32, "fp64": adj64, "rel_diff_vs_forward_fp64": adj_sym},
            "z_step_fp32": {"ms": zms, "tflops": zflops / (zms * 1e-3) / 1e12,
                            "kernel": "k_zdirect5m (v_mfma_f32_16x16x4f32)" if zflops_mfma else "k_zdirect5 (VALU)",
                            "mfma_tflops_executed": zflops_mfma / (zms * 1e-3) / 1e12 if zflops_mfma else None,
                            "mfma_frac": (zflops_mfma / (zms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS) if zflops_mfma else None,
                            "alu_frac": None if zflops_mfma else zflops / (zms * 1e-3) / 1e12 / FP32_VALU_PEAK_TFLOPS,
                            "hbm_gbs": by["pass_z_mul"] / (zms * 1e-3) / 1e9}}


def bench_table2(args):
    """Table II (Sec. III.B.3) on synthetic cubes of edge n voxels (dx = 1 um):
    the seven unit-voxel tables computed directly (device quadrature) against
    restored from an Algorithm 2 store (Tucker tol 1e-8, built once for the
    largest cube, as at installation), with their memory."""
    import tempfile
    import torch
    import paper_2105_08627_amd as svh
    sizes = [int(v) for v in args.table2.split(",")]
    big = max(sizes)
    path = os.path.join(tempfile.mkdtemp(), "store.svh")
    t = time.perf_counter()
    err = svh.toeplitz_store_build((big, big, big), 7, 1e-8, path)
    t_build = time.perf_counter() - t
    log(f"[bench] table2 store {big}^3 built in {t_build:.1f}s, {os.path.getsize(path) / 2**20:.2f} MB")
    rows = []
    for n in sizes:
        buf = torch.empty(7 * n ** 3, dtype=torch.float64, device="cuda")
        ref = torch.empty_like(buf)
        svh.green_tables((n, n, n), 7, ref)  # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        svh.green_tables((n, n, n), 7, ref)
        torch.cuda.synchronize()
        t_direct = time.perf_counter() - t
        svh.toeplitz_store_restore(path, (n, n, n), 7, buf)
        torch.cuda.synchronize()
        t = time.perf_counter()
        svh.toeplitz_store_restore(path, (n, n, n), 7, buf)
        torch.cuda.synchronize()
        t_restore = time.perf_counter() - t
        rel = (torch.linalg.vector_norm(buf - ref) / torch.linalg.vector_norm(ref)).item()
        row = {"edge_voxels": n, "tables_MB": 7 * n ** 3 * 8 / 2 ** 20, "store_MB": os.path.getsize(path) / 2 ** 20,
               "direct_s": t_direct, "restore_s": t_restore, "restore_relerr": rel}
        log(f"[bench] table2 {row}")
        rows.append(row)
        del buf, ref
    os.remove(path)
    return {"store_domain": big, "store_build_s": t_build, "store_relerr_bound": err, "rows": rows}


def bench_tucker_sweep(args):
    """Figs. 2-3 (Sec. III.B.1) on synthetic cubes (3D) and 3-voxel plates
    (2D-like), dx = 1 um: multilinear ranks of the circulant spectrum, the
    compression ratio CR (dense circulant bytes / Tucker bytes) and the
    overhead CO (restoration time / one convolution of one component with the
    same tensor, both on the device, FP32 product) per Tucker tolerance."""
    import torch
    import paper_2105_08627_amd as svh
    dev = torch.device("cuda:0")
    rows = []
    shapes = [(n, n, n) for n in (32, 64, 100, 128, 192, 256)] + [(n, n, 3) for n in (128, 256, 384, 512)]
    for K in shapes:
        mask = np.ones(K[::-1], dtype=np.uint8)
        p = svh.Problem(mask, 1e-6)
        p.set_material([1e9], 0.0, 90e-9)
        p.setup_tensors()
        x = torch.from_numpy(np.ones((1, 3, p.K), dtype=np.complex64)).to(dev)
        Lt = p.L[0] * p.L[1] * p.L[2]
        for tol in (1e-4, 1e-6, 1e-8):
            ranks, err = p.tucker_compress(tol)
            d1, d2, d3 = ranks
            tucker_bytes = 8 * (d1 * d2 * d3 + p.L[0] * d1 + p.L[1] * d2 + p.L[2] * d3)
            p.matvec(x, [-1])
            torch.cuda.synchronize()
            p.profile(True)
            p.profile_read()
            for _ in range(5):
                p.matvec(x, [-1])
            prof, n = p.profile_read()
            p.profile(False)
            conv = sum(v for k, v in prof.items() if k != "tucker_restore") / (3 * n)
            rows.append({"shape": list(K), "Kt": int(np.prod(K)), "tol": tol, "ranks": list(ranks),
                         "CR": Lt * 8 / tucker_bytes, "CO": prof["tucker_restore"] / n / conv,
                         "tucker_MB": tucker_bytes / 2 ** 20, "dense_MB": Lt * 8 / 2 ** 20})
            log(f"[bench] tucker sweep {rows[-1]}")
        del p
    return {"rows": rows}


def bench_bend_study(args):
    """Self-convergence of the 90-degree bend inductance (Sec. III.C geometry:
    2 x 2 mm square section, 10 mm arms, lambda = 0.45 mm, sigma0 = 0) with the
    piecewise-linear basis at dx = 0.5, 0.4, 0.25, 0.2, 0.1, 0.05 and
    0.025 mm (the paper's two finest; their 40 and 80 planes take the z FFT
    step); the finest grid is the reference."""
    import torch
    import paper_2105_08627_amd as svh
    import workloads as wl
    f = 1e3
    res = []
    for dx_mm in (0.5, 0.4, 0.25, 0.2, 0.1, 0.05, 0.025):
        mask, ports = wl.square_bend(int(round(2.0 / dx_mm)), int(round(10.0 / dx_mm)))
        t = time.perf_counter()
        p = svh.Problem(mask, dx_mm * 1e-3, basis=5)
        p.set_material([f], 0.0, 0.45e-3)
        p.setup_tensors()
        p.tucker_compress(1e-8)
        p.set_ports(ports)
        t_setup = time.perf_counter() - t
        t = time.perf_counter()
        X, Y, info = p.solve(0, rre=1e-8, restart=50, maxit=2000)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        L = float(p.port_inductance(0, Y)[1][0, 0])
        nz = int(np.count_nonzero(mask.reshape(mask.shape[0], -1).any(axis=1)))
        res.append({"dx_mm": dx_mm, "grid": list(mask.shape[::-1]), "occupied_planes": nz, "K": p.K, "N": p.N,
                    "L_nH": L * 1e9, "iterations": info["iterations"], "setup_s": t_setup, "solve_s": dt,
                    "relres": info["relres"]})
        log(f"[bench] bend {res[-1]}")
        del p, X
    ref = res[-1]["L_nH"]
    for r in res:
        r["rel_diff_vs_finest"] = abs(r["L_nH"] - ref) / abs(ref)
    return {"frequency_hz": f, "rows": res}


def bench_solve(args):
    """Port solve (eq. 7) of 16 coupled strips (256 x 128 x 4 grid, 16 ports),
    plain FP64 vs FP32 products inside FP64 refinement, both to relative
    residual 1e-8 (the paper's setting), restart 50."""
    import torch
    import paper_2105_08627_amd as svh
    import workloads as wl
    mask, ports = wl.strip_array()
    dx, f = 0.25e-6, 10e9
    p = svh.Problem(mask, dx)
    p.set_material([f], 1e7, 90e-9)
    p.setup_tensors()
    p.tucker_compress(1e-8)
    p.set_ports(ports)
    log(f"[bench] solve workload: strips K={p.K} N={p.N} ports={len(ports)}")
    res = {}
    for name, refine in (("fp64", False), ("fp32_refined", True)):
        p.solve(0, rre=1e-8, restart=50, refine=refine)  # warm-up (graphs, caches)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, Y, info = p.solve(0, rre=1e-8, restart=50, refine=refine)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[name] = {"seconds": dt, "Y": Y, **{k: info[k] for k in ("iterations", "inner_iterations",
                                                                     "refinement_steps", "relres")}}
        log(f"[bench] solve {name}: {dt:.3f}s {info['iterations']} its, inner {info['inner_iterations']}, "
            f"relres {info['relres']:.2e}")
    Y64, Yir = res["fp64"].pop("Y"), res["fp32_refined"].pop("Y")
    res["gradient"] = bench_gradient(p, f)
    return {"workload": f"16 coupled strips {mask.shape[2]}x{mask.shape[1]}x{mask.shape[0]}, K={p.K}, "
                        f"N={p.N} per port, 16 ports, rre 1e-8", **res,
            "admittance_rel_diff_fp32_refined_vs_fp64": float(np.abs(Yir - Y64).max() / np.abs(Y64).max())}


def bench_solve_strips_over_ground(args):
    """Port solve of the 128 x 128 x 64 strips-over-ground workload: 16 ports
    in one batch, piecewise-linear basis (five components, so current turns
    the vias' corners), Tucker tol 1e-6, FP32 products in FP64 refinement and
    plain FP64, both to relative residual 1e-8."""
    import torch
    import paper_2105_08627_amd as svh
    import workloads as wl
    mask, ports = wl.strips_over_ground_with_ports(1002)
    f = 10e9
    p = svh.Problem(mask, 0.25e-6, basis=5)
    p.set_material([f], 1e7, 90e-9)
    p.setup_tensors()
    p.tucker_compress(1e-6)
    p.set_ports(ports)
    res = {}
    for name, refine in (("fp32_refined", True), ("fp64", False)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, Y, info = p.solve(0, rre=1e-8, restart=50, refine=refine)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[name] = {"seconds": dt, "Y": Y, **{k: info[k] for k in ("iterations", "inner_iterations",
                                                                     "refinement_steps", "relres")}}
        log(f"[bench] strips-over-ground solve {name}: {dt:.2f}s {info['iterations']} its, "
            f"inner {info['inner_iterations']}, relres {info['relres']:.2e}")
        del X
    # reference admittance: FP64 to relative residual 1e-11 (untimed)
    _, Yref, iref = p.solve(0, rre=1e-11, restart=50, maxit=3000)
    Y64, Yir = res["fp64"].pop("Y"), res["fp32_refined"].pop("Y")
    for name, Yv in (("fp64", Y64), ("fp32_refined", Yir)):
        res[name]["admittance_rel_err_vs_reference"] = float(np.abs(Yv - Yref).max() / np.abs(Yref).max())
    return {"workload": f"strips over a ground slab with 16 holes, {mask.shape[2]}x{mask.shape[1]}x{mask.shape[0]}, "
                        f"K={p.K}, five components, N={p.N} per port, 16 ports, rre 1e-8, Tucker tol 1e-6",
            **res, "admittance_rel_diff_fp32_refined_vs_fp64": float(np.abs(Yir - Y64).max() / np.abs(Y64).max()),
            "reference": f"FP64 solve to relative residual {iref['relres']:.1e} ({iref['iterations']} iterations)"}


def bench_c5_solve(args):
    """Port solve of the 256 x 256 x 128 stack with its 8 port-gap vias
    (five components, so current turns the vias' corners; 52 occupied planes,
    so the z FFT step), 8 ports in one batch, at the lowest and the highest of
    the 8 frequencies: FP32 products inside FP64 refinement against plain
    FP64, both to relative residual 1e-8, Tucker tol 1e-8."""
    import torch
    import paper_2105_08627_amd as svh
    import workloads as wl
    cfg = wl.WORKLOADS["c5_stack"]
    mask, ports = wl.layered_stack_with_ports(cfg["seed"])
    freqs = [cfg["freqs"][0], cfg["freqs"][-1]]
    if args.c5_freq >= 0:
        freqs = [freqs[args.c5_freq]]
    t = time.perf_counter()
    p = svh.Problem(mask, cfg["dx"], basis=5)
    p.set_material(freqs, cfg["sigma0"], cfg["lam"])
    p.setup_tensors()
    ranks, _ = p.tucker_compress(1e-8)
    p.set_ports(ports)
    t_setup = time.perf_counter() - t
    log(f"[bench] c5 solve: K={p.K} N={p.N} ports={len(ports)} setup {t_setup:.1f}s")
    rows = []
    for fi, f in enumerate(freqs):
        res = {"frequency_hz": f}
        for name, refine in (("fp32_refined", True), ("fp64", False)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            X, Y, info = p.solve(fi, rre=1e-8, restart=50, maxit=2000, refine=refine, check=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            res[name] = {"seconds": dt, "Y": Y, **{k: info[k] for k in ("iterations", "inner_iterations",
                                                                         "refinement_steps", "relres", "converged")}}
            log(f"[bench] c5 solve f={f:.3g} {name}: {dt:.2f}s {info['iterations']} its, "
                f"inner {info['inner_iterations']}, relres {info['relres']:.2e}")
            del X
        Y64, Yir = res["fp64"].pop("Y"), res["fp32_refined"].pop("Y")
        res["admittance_rel_diff_fp32_refined_vs_fp64"] = float(np.abs(Yir - Y64).max() / np.abs(Y64).max())
        Z, L = p.port_inductance(fi, Y64)
        res["port_self_inductance_pH"] = (np.diag(L) * 1e12).tolist()
        rows.append(res)
    return {"workload": f"stack with 8 port-gap vias, {mask.shape[2]}x{mask.shape[1]}x{mask.shape[0]}, K={p.K}, "
                        f"five components, N={p.N} per port, 8 ports, rre 1e-8, Tucker tol 1e-8",
            "setup_s": t_setup, "tucker_ranks": ranks.tolist(), "rows": rows}


def bench_gradient(p, f):
    """Gradient of the full port-inductance matrix with respect to every
    voxel's lambda^-2 (addition 3): forward solve, adjoint solve (transpose),
    per-voxel admittance derivative, contraction with the loss weights
    G = all ones (the library forms W = Z^T G Z^T).  Timed after one untimed
    pass."""
    import torch
    for timed in (False, True):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, Y, _ = p.solve(0, rre=1e-8, restart=50)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        Xa, _, info = p.solve(0, rre=1e-8, restart=50, transpose=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        # the two short steps are timed as the median of 5 calls each: the
        # first host call into the library after a solve has been seen to
        # take about 14 ms whatever it does (host-only calls included)
        tg, tc = [], []
        for _ in range(5):
            ta = time.perf_counter()
            dY = p.port_gradient(0, X, Xa)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            g = p.gradient_contract(0, Y, np.ones(Y.shape), dY)
            torch.cuda.synchronize()
            tg.append(tb - ta)
            tc.append(time.perf_counter() - tb)
        t4 = time.perf_counter()
    mg, mc = float(np.median(tg)), float(np.median(tc))
    log(f"[bench] gradient: forward {t1 - t0:.3f}s adjoint {t2 - t1:.3f}s ({info['iterations']} its) "
        f"dY {1e3 * mg:.2f} ms contract {1e3 * mc:.2f} ms (medians of 5; first calls {1e3 * tg[0]:.2f}, "
        f"{1e3 * tc[0]:.2f} ms)")
    return {"what": "d(sum of all port inductances)/d(lambda_k^-2) for every voxel k, FP64, rre 1e-8",
            "forward_solve_s": t1 - t0, "adjoint_solve_s": t2 - t1, "adjoint_iterations": info["iterations"],
            "port_gradient_ms": 1e3 * mg, "contract_ms": 1e3 * mc, "first_call_ms": [1e3 * tg[0], 1e3 * tc[0]],
            "total_s": (t2 - t0) + mg + mc,
            "dY_entries": int(dY.numel()), "grad_finite": bool(torch.isfinite(g).all().item())}


def bench_adjoint(p, x, fidx, steps):
    """Adjoint product y = Z^T x (addition 3) on the same batch as the
    forward product, timed like it."""
    import torch
    y = torch.empty_like(x)
    p.matvec_adjoint(x, fidx, out=y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        p.matvec_adjoint(x, fidx, out=y)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return y, {"ms_per_step": dt * 1e3 / steps, "matvecs_per_s": x.shape[0] * steps / dt}


def bench_matvec(args, dev):
    """The headline section: the batched product on the stack (or the
    workload named), FP32 and FP64, adjoint, roofline; then the same grid with
    five components."""
    import torch
    import paper_2105_08627_amd as svh
    import workloads as wl
    cfg = wl.WORKLOADS[args.workload]
    mask = cfg["mask"]()
    dx, freqs, sigma0, lam = cfg["dx"], cfg["freqs"], cfg["sigma0"], cfg["lam"]
    nrhs = args.nrhs
    nf = len(freqs)
    fidx = [r % nf for r in range(nrhs)]
    log(f"[bench] workload {args.workload} grid {mask.shape[::-1]} K={int(mask.sum())} nrhs={nrhs}")
    t = time.perf_counter()
    p = svh.Problem(mask, dx)
    p.set_material(freqs, sigma0, lam)
    p.setup_tensors()
    p.set_zstep(args.zstep)
    t_setup = time.perf_counter() - t
    t = time.perf_counter()
    ranks, terr = p.tucker_compress(args.tol)
    t_tucker = time.perf_counter() - t
    log(f"[bench] setup {t_setup:.1f}s tucker {t_tucker:.1f}s  L={p.L} tucker ranks {ranks} bound {terr:.2e}")
    K = p.K
    nzp = int(np.count_nonzero(mask.reshape(mask.shape[0], -1).any(axis=1)))
    x64_h = wl.random_currents(cfg["seed"], (nrhs, 3, K))
    x64 = torch.from_numpy(x64_h).to(dev)
    x32 = x64.to(torch.complex64)
    y32 = torch.empty_like(x32)
    y64 = torch.empty_like(x64)
    torch.cuda.synchronize()

    # autotune the launch shapes on this batch (both precisions)
    t = time.perf_counter()
    ms32 = p.autotune(x32, fidx)
    ms64 = p.autotune(x64, fidx)
    log(f"[bench] autotune {time.perf_counter() - t:.1f}s: tuned kernel ms fp32 {ms32:.3f} fp64 {ms64:.3f}")

    # FP32 (production path), timed
    for _ in range(args.warmup):
        p.matvec(x32, fidx, out=y32)
    torch.cuda.synchronize()
    p.profile(True)
    p.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        p.matvec(x32, fidx, out=y32)
    torch.cuda.synchronize()
    dt32 = time.perf_counter() - t0
    prof32, ncall = p.profile_read()
    p.profile(False)
    log(f"[bench] fp32 {args.steps} steps {dt32 * 1e3 / args.steps:.3f} ms/step  per-kernel ms/call "
        + " ".join(f"{k}={v / args.steps:.3f}" for k, v in prof32.items()))

    # FP64 path
    for _ in range(1):
        p.matvec(x64, fidx, out=y64)
    torch.cuda.synchronize()
    p.profile(True)
    p.profile_read()
    t0 = time.perf_counter()
    for _ in range(args.fp64_steps):
        p.matvec(x64, fidx, out=y64)
    torch.cuda.synchronize()
    dt64 = time.perf_counter() - t0
    prof64, ncall64 = p.profile_read()
    p.profile(False)
    log(f"[bench] fp64 {args.fp64_steps} steps {dt64 * 1e3 / args.fp64_steps:.3f} ms/step")
    rel = (torch.linalg.vector_norm((y32.to(torch.complex128) - y64).flatten())
           / torch.linalg.vector_norm(y64.flatten())).item()

    # adjoint product (same kernels through the transposed block table)
    ya32, adj32 = bench_adjoint(p, x32, fidx, max(args.steps // 2, 1))
    ya64, adj64 = bench_adjoint(p, x64, fidx, args.fp64_steps)
    adj_sym = (torch.linalg.vector_norm((ya64 - y64).flatten()) / torch.linalg.vector_norm(y64.flatten())).item()
    del ya32, ya64
    log(f"[bench] adjoint fp32 {adj32['ms_per_step']:.3f} ms/step fp64 {adj64['ms_per_step']:.3f} ms/step "
        f"|Z^T x - Z x|/|Z x| {adj_sym:.1e}")

    mv32 = nrhs * args.steps / dt32
    mv64 = nrhs * args.fp64_steps / dt64
    nvec = 3 * nrhs
    zocc = np.flatnonzero(mask.reshape(mask.shape[0], -1).any(axis=1))
    nd = len({abs(int(a) - int(b)) for a in zocc for b in zocc})
    by32 = pass_bytes(p, nvec, 8, 4, K, nzp, nd)
    per_call = {k: v / args.steps for k, v in prof32.items()}
    dom = max(by32, key=lambda k: per_call[k])
    ach = by32[dom] / (per_call[dom] * 1e-3) / 1e9
    total_bytes = sum(by32.values())
    kern_ms = sum(per_call[k] for k in by32)
    # Tucker restoration: FLOPs of the three mode products
    d1, d2, d3 = ranks
    Lx, Ly, Lz = p.L
    # the direct z step restores the distinct plane offsets only
    tflops = 2.0 * (Lx * d1 * d2 * d3 + Lx * Ly * d2 * d3 + Lx * Ly * (nd if nzp <= 32 else Lz) * d3)
    tk_ms = per_call["tucker_restore"]
    out = {
        "metric": "FFT-VIE matvecs/s (FP32 operator inside FP64 refinement; FP64 beside it)",
        "value": mv32,
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt32 * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (FFT, product); f64 Tucker restoration",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {mask.shape[2]}x{mask.shape[1]}x{mask.shape[0]} grid, "
                               f"K={K} voxels, 3 components, {nrhs} RHS (8 ports x {nf} frequencies), "
                               f"Tucker tol {args.tol:g}",
                   "fft_grid": list(p.L), "tucker_ranks": list(ranks), "occupied_z_planes": nzp},
        "setup_s": {"green_tables_and_spectrum": t_setup, "tucker_compress": t_tucker},
        "fp64": {"value": mv64, "unit": "matvecs/s", "ms_per_step": dt64 * 1e3 / args.fp64_steps},
        "rel_err_fp32_vs_fp64": rel,
        "voxel_matvecs_per_s": {"fp32_Kt": mv32 * mask.size, "fp32_K": mv32 * K,
                                "fp64_Kt": mv64 * mask.size},
        "kernels_ms_per_step": per_call,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": measured_traffic(KERNEL_NAMES_FP32.get(dom)),
                     "all_passes_frac": total_bytes / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "adjoint": {"fp32": adj32, "fp64": adj64, "rel_diff_vs_forward_fp64": adj_sym},
        "tucker_restore": {"ms": tk_ms, "tflops": tflops / (tk_ms * 1e-3) / 1e12 if tk_ms > 0 else None,
                           "mfma_frac": (tflops / (tk_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS) if tk_ms > 0 else None},
    }
    if not args.no_basis5:
        out["basis5"] = bench_basis5(args, cfg, mask, fidx, dev)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c5_stack")
    ap.add_argument("--nrhs", type=int, default=64)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-strips", action="store_true", help="skip the 16-strip solve (keep strips over ground)")
    ap.add_argument("--no-basis5", action="store_true")
    ap.add_argument("--tucker-sweep", action="store_true", help="ranks, CR and CO vs domain size (Figs. 2-3)")
    ap.add_argument("--bend-study", action="store_true", help="90-degree bend inductance vs voxel size")
    ap.add_argument("--c5-solve", action="store_true",
                    help="port solve of the stack with its 8 port-gap vias (five components)")
    ap.add_argument("--no-matvec", action="store_true", help="skip the matvec sections (with --c5-solve etc.)")
    ap.add_argument("--c5-freq", type=int, default=-1,
                    help="with --c5-solve: 0 = lowest frequency only, 1 = highest only (default both)")
    ap.add_argument("--table2", default="",
                    help="comma-separated cube edges (voxels) for the Toeplitz-store experiment, e.g. 100,200")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--zstep", default="auto", choices=["auto", "fft", "direct", "fused"])
    ap.add_argument("--cpu-worker", default="", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-rows", type=int, default=2048, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-budget", type=float, default=20.0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker:
        cpu_worker(args.cpu_worker, args.nrhs, args.cpu_rows, args.cpu_budget)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU sharding is not built "
                                   "(--gpus must be 1)"}))
        sys.exit(2)
    # the CPU baselines' child process starts before anything touches the GPU
    cpu = None if args.no_cpu else CpuBaseline(args.workload, args.nrhs)

    import torch

    dev = torch.device("cuda:0")
    if args.copy_probe:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev).fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    out = {} if args.no_matvec else bench_matvec(args, dev)
    if not args.no_solve:
        if not args.no_strips:
            out["solve"] = bench_solve(args)
        out["solve_strips_over_ground"] = bench_solve_strips_over_ground(args)
    if args.table2:
        out["table2"] = bench_table2(args)
    if args.tucker_sweep:
        out["tucker_sweep"] = bench_tucker_sweep(args)
    if args.bend_study:
        out["bend_study"] = bench_bend_study(args)
    if args.c5_solve:
        out["c5_solve"] = bench_c5_solve(args)
    if cpu is not None:
        log("[bench] cpu baselines (oracle row sum, scipy.fft product) ...")
        cb = cpu.result()
        out["cpu_baseline"] = cb["dense"]
        out["cpu_fft_baseline"] = cb["fft"]
        log(f"[bench] cpu {cb}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
