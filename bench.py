"""Benchmark: the node sweep of the contour rational approximation on one MI355X.

Workload "sphere-81920" (the headline configuration): unit icosphere at subdivision level
6 (n = 81920 flat triangles, P0 collocation at centroids, single-layer kernel
exp(i kappa r)/(4 pi r), 7-point rule plus exact self terms), circular contour
|z - 5| = 2 with N = 64 trapezoidal nodes, probe block of m = 64 seeded complex Gaussian
columns (seed 2).  One step = the nodes and moment weights (host) plus one rr_project
call with fused moments in the per-node (direct) form: every operator T(z_j) regenerated
and contracted with the probe block, i.e. all N n^2 m complex multiply-adds, giving the
projections U^H T(z_j) U for all 64 nodes and the first P = 2 contour moments
sum_j w_j (z_j - c)^-p T(z_j) U; self terms, sweep, combination and projection all run on
the device.

Metric: kernel-entry x RHS per second, N n^2 m / t_step, t_step the device time of one step.
Beside it ("taylor_form") the same call in the Taylor-expansion form, which generates and
contracts L < N coefficient operators and recombines them per node: its rate in the same
units is an effective one (N n^2 m / t), reported with the L n^2 m entries it contracts.

Prints one JSON line (see the repository's design notes for every field).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_MFMA_TFLOPS = 78.6  # MI355X published dense FP64 matrix peak
WORKLOAD = dict(name="sphere-81920", level=6, c=5.0, radius=2.0, N=64, m=64, P=2, seed=2)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("sweep.hip", "generators.h", "devmath.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_1906_03938_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(name: str, kernel_hash: str):
    """HBM bytes per launch measured by rocprofv3 --pmc (FETCH_SIZE, WRITE_SIZE) for the kernel
    summarised in profiles/<name>, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash:
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(xyz, tri, z, V, rows=256):
    """The oracle (plain FP64 C, OpenMP over target rows) on a bounded sample: the full
    N-node sweep of T(z_j) V for a fixed slice of `rows` target rows spread evenly over the
    mesh (all sources, all probe columns), scaled to entry x RHS per second."""
    import numpy as np

    from oracle import _clib

    threads = _clib.num_threads()
    n = tri.shape[0]
    sel = np.linspace(0, n - 1, rows).astype(np.int64)
    t0 = time.perf_counter()
    for zj in z:
        _clib.apply_rows(xyz, tri, zj, V, sel)
    dt = time.perf_counter() - t0
    units = sel.size * n * len(z) * V.shape[1]
    return {
        "value": units / dt,
        "unit": "kernel-entry*RHS/s",
        "cores": int(min(threads, sel.size)),
        "kind": "oracle",
        "sample": f"{sel.size} of {n} target rows (evenly spaced) x all {n} source triangles x {len(z)} nodes x "
                  f"{V.shape[1]} probes ({dt:.1f} s), scaled by entry*RHS count; the full sweep would be "
                  f"{n / sel.size:.0f}x this sample",
    }


PRECISION_WORKLOAD = dict(name="box-119912", dims=(1.0, 0.8, 0.6), counts=(126, 101, 76), a=2.0, b=8.0, N=48,
                          m=128, seed=3)
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "f16": 2500.0}  # MI355X dense matrix peaks


def precision_sweeps():
    """Only the timed sweeps of precision_form (the four cheb_moments calls on box-119912, no
    eigen-solves): a short command for the reduced-precision kernels' counters."""
    return precision_form(eigen=False)


def precision_form(eigen=True):
    """The precision form on the box workload (1.0 x 0.8 x 0.6 box, 126 x 101 x 76 face grid,
    n = 119,912; Chebyshev blocks on [2, 8] with N = 48 nodes, m = 128 probes, seed 3): one
    cheb_moments call per arithmetic after a warm-up call at FP64, timed by the library's
    events around its sweep kernel (and wall clock for the whole call), and the eigenvalue
    error per arithmetic on the 752-triangle box (interval [6.5, 8], N = 24), with every
    sweep at that arithmetic ("all") and with FP64 Rayleigh-Ritz projections ("rr_f64"),
    against the oracle's value in tests/golden/box752_interval_eigs.txt."""
    import numpy as np
    import torch

    import paper_1906_03938_amd as bem
    import synth
    from paper_1906_03938_amd.eig import eigs_in_interval

    w = PRECISION_WORKLOAD
    xyz, tri = synth.box_surface(w["dims"], w["counts"])
    n = tri.shape[0]
    V = torch.from_numpy(synth.probe_block(n, w["m"], seed=w["seed"])).to("cuda")
    precs = (("f64", bem.PREC_F64), ("f32", bem.PREC_F32), ("bf16", bem.PREC_BF16), ("f16", bem.PREC_F16))
    forms = {}
    with bem.Mesh(xyz, tri) as mesh:
        mesh.set_timing(True)
        mesh.cheb_moments(w["a"], w["b"], w["N"], w["N"], V)  # warm-up (workspace)
        torch.cuda.synchronize()
        for name, p in precs:
            t0 = time.perf_counter()
            mesh.cheb_moments(w["a"], w["b"], w["N"], w["N"], V, form=bem.FORM_AUTO | p)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            kms = mesh.last_kernel_ms()
            form, L = mesh.last_form()
            fl = 8.0 * L * n * n * w["m"]
            forms[name] = {"value": w["N"] * n * n * w["m"] / wall, "unit": "kernel-entry*RHS/s",
                           "seconds": wall, "sweep_kernel_ms": kms,
                           "form": {bem.FORM_DIRECT: "direct", bem.FORM_EXPAND: "expand",
                                    bem.FORM_CHEB: "cheb"}[form], "operators_generated": L,
                           "achieved_tflops": fl / (kms * 1e-3) / 1e12, "matrix_peak_tflops": PEAK_TFLOPS[name]}
    base = forms["f64"]["value"]
    for name in forms:
        forms[name]["speedup_vs_f64"] = forms[name]["value"] / base
    if not eigen:
        return {"workload": w["name"], "forms": forms}
    ref = np.loadtxt(os.path.join(ROOT, "tests", "golden", "box752_interval_eigs.txt"))
    lam_ref = ref[0] + 1j * ref[1]
    bx, bt = synth.box_surface(w["dims"], (10, 8, 6))
    U0 = synth.probe_block(bt.shape[0], 8, seed=3)
    eig = {}
    with bem.Mesh(bx, bt) as mesh:
        for name, p in precs:
            for mode in ("all", "rr_f64"):
                if name == "f64" and mode == "rr_f64":
                    continue
                lam, _, res, outer = eigs_in_interval(mesh, 6.5, 8.0, 24, U0, q=10, tol=1e-12, max_outer=4,
                                                      sweep_prec=p, rr_prec=p if mode == "all" else bem.PREC_F64)
                err = float(np.max(np.abs(lam - lam_ref)) / abs(lam_ref)) if lam.size == 1 else None
                eig[f"{name}/{mode}"] = {"rel_err": err, "found": int(lam.size),
                                         "max_rel_residual": float(res.max()) if res.size else None,
                                         "outer_iterations": int(outer)}
    return {"workload": w["name"], "mesh": f"box 1.0x0.8x0.6, face grid 126x101x76, n={n}",
            "interval": [w["a"], w["b"]], "nodes": w["N"], "m": w["m"], "call": "cheb_moments, all N blocks",
            "forms": forms, "eigen_box752": eig, "equal_accuracy": equal_accuracy()}


def equal_accuracy(counts=(50, 40, 30)):
    """The whole interval eigen-solve (Chebyshev route, [6.5, 8], N = 24, 8 probes, seed 3, q = 10)
    on the 1.0 x 0.8 x 0.6 box of 4 (nx ny + nx nz + ny nz) triangles (n = 18,800 for the
    default grid) with every sweep in FP64, and with the subspace sweeps in FP32 or BF16 and
    the Rayleigh-Ritz projections in FP64, each stopped at relative residual 1e-6; the
    eigenvalue error of each against an FP64 solve stopped at 1e-12, and the wall time of each
    solve (G assembled and factorised on the device included)."""
    import numpy as np
    import torch

    import paper_1906_03938_amd as bem
    import synth
    from paper_1906_03938_amd.eig import eigs_in_interval

    xyz, tri = synth.box_surface((1.0, 0.8, 0.6), counts)
    n = tri.shape[0]
    U0 = synth.probe_block(n, 8, seed=3)
    out = {"mesh": f"box 1.0x0.8x0.6, face grid {counts[0]}x{counts[1]}x{counts[2]}, n={n}",
           "interval": [6.5, 8.0], "nodes": 24, "probes": 8, "tol": 1e-6, "runs": {}}
    with bem.Mesh(xyz, tri) as mesh:
        lam_ref, _, _, _ = eigs_in_interval(mesh, 6.5, 8.0, 24, U0, q=10, tol=1e-12, max_outer=8)
        out["reference_eigenvalues"] = [[float(l.real), float(l.imag)] for l in lam_ref]
        for name, sp in (("f64", bem.PREC_F64), ("f32_sweeps_f64_rr", bem.PREC_F32),
                         ("bf16_sweeps_f64_rr", bem.PREC_BF16)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lam, _, res, outer = eigs_in_interval(mesh, 6.5, 8.0, 24, U0, q=10, tol=1e-6, max_outer=8, sweep_prec=sp,
                                                  rr_prec=bem.PREC_F64)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            err = (float(np.max(np.abs(np.sort_complex(lam) - np.sort_complex(lam_ref)) / np.abs(lam_ref)))
                   if lam.size == lam_ref.size else None)
            out["runs"][name] = {"seconds": t, "found": int(lam.size), "rel_err_vs_f64_1e-12": err,
                                 "max_rel_residual": float(res.max()) if res.size else None,
                                 "outer_iterations": int(outer)}
    f64 = out["runs"]["f64"]["seconds"]
    for r in out["runs"].values():
        r["speedup_vs_f64"] = f64 / r["seconds"]
    return out


BATCH_WORKLOAD = dict(name="ellipsoids-64", count=64, seed=4, freq=(10, 44), axes=(0.5, 1.5), centre=(3.0, 7.0),
                      radius=1.0, N=32, m=32, P=2)


def batched_form():
    """The batched persistent form on 64 seeded ellipsoids (class-I geodesic frequencies
    10..44, i.e. 2,000-38,720 triangles, semi-axes in [0.5, 1.5], seed 4), each with its
    own circle |z - c_i| = 1, c_i in [3, 7], N = 32 nodes, P = 2 moments and m = 32 probes
    (seeds 4000 + i): one bem_batch_moments call (after the batch's set-up with the tile
    autotuner and one warm-up call), timed by wall clock and by the library's events around
    the persistent kernel, beside the same moments by 64 per-mesh contour_moments calls in
    the same form on the same stream (the batch and these calls both fold the two weight sets
    into the sweep), and the batch with an FP32 contraction (autotuned; the
    direct form that AUTO takes at reduced precision, and the expansion form on request) with
    its error against the FP64 result."""
    import numpy as np
    import torch

    import paper_1906_03938_amd as bem
    import synth

    w = BATCH_WORKLOAD
    spec = synth.ellipsoid_batch(count=w["count"], seed=w["seed"], freq=w["freq"], axes=w["axes"],
                                 centre=w["centre"])
    sizes = np.array([t.shape[0] for _, t, _, _ in spec], dtype=np.float64)
    meshes = [bem.Mesh(x, t) for x, t, _, _ in spec]
    z, W = [], []
    for _, _, _, c in spec:
        zi, _, Wi = bem.contour_nodes(c, w["radius"], w["N"], P=w["P"])
        z.append(zi)
        W.append(Wi)
    z, W = np.array(z), np.array(W)
    V = [synth.probe_block(int(n), w["m"], seed=4000 + i) for i, n in enumerate(sizes)]
    Vd = torch.from_numpy(np.concatenate(V, axis=0)).to("cuda")
    t0 = time.perf_counter()
    batch = bem.Batch(meshes, z, W, w["m"], tune=True)
    setup = time.perf_counter() - t0
    batch.set_timing(True)
    out = torch.empty(w["P"] * int(batch.rows[-1]) * w["m"], dtype=torch.complex128, device="cuda")
    batch.moments(Vd, out=out)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.moments(Vd, out=out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = batch.last_kernel_ms()
    eager_out = out.clone()
    L = batch.operators.astype(np.float64)
    units = float(np.sum(w["N"] * sizes ** 2 * w["m"]))
    # an FP64 batch with up to four weight sets folds them into the sweep (every operator of
    # an entry generated, only the P folds contracted), as contour_moments does per mesh
    folded = w["P"] <= 4
    flops = float(np.sum(8.0 * (w["P"] if folded else L) * sizes ** 2 * w["m"]))
    achieved = flops / (kms * 1e-3) / 1e12
    # the same call captured once in a HIP graph (the path a serving loop takes) and replayed;
    # timing events are off so the capture holds only the call's own kernels
    batch.set_timing(False)
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        batch.moments(Vd, out=out)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(cs)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.moments(Vd, out=out)
    graph.replay()
    torch.cuda.synchronize()
    replay_ms = []
    for _ in range(2):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        graph.replay()
        e1.record()
        e1.synchronize()
        replay_ms.append(e0.elapsed_time(e1))
    graph_ms = float(np.median(replay_ms))
    graph_equal = bool(torch.equal(out, eager_out))
    batch.set_timing(True)
    # the same moments by one call per mesh
    Vs = [torch.from_numpy(v).to("cuda") for v in V]
    outs = [torch.empty((w["P"], int(n), w["m"]), dtype=torch.complex128, device="cuda") for n in sizes]
    for i, mesh in enumerate(meshes):  # warm-up (workspaces)
        mesh.contour_moments(z[i], W[i], Vs[i], out=outs[i], form=batch.form)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, mesh in enumerate(meshes):
        mesh.contour_moments(z[i], W[i], Vs[i], out=outs[i], form=batch.form)
    torch.cuda.synchronize()
    wall_seq = time.perf_counter() - t0
    parts = batch.split(out)
    diff = max(float(torch.linalg.vector_norm(parts[i] - outs[i]) / torch.linalg.vector_norm(outs[i]))
               for i in range(len(meshes)))
    # FP32 contraction (AUTO at reduced precision: the direct form), against the FP64 result
    lp = {}
    for name, flags in (("f32", bem.FORM_AUTO | bem.PREC_F32), ("f32_expand", bem.FORM_EXPAND | bem.PREC_F32)):
        b32 = bem.Batch(meshes, z, W, w["m"], form=flags, tune=True)
        b32.set_timing(True)
        o32 = torch.empty_like(out)
        b32.moments(Vd, out=o32)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b32.moments(Vd, out=o32)
        torch.cuda.synchronize()
        wall32 = time.perf_counter() - t0
        k32 = b32.last_kernel_ms()
        p32 = b32.split(o32)
        err = max(float(torch.linalg.vector_norm(p32[i][q] - parts[i][q]) / torch.linalg.vector_norm(parts[i][q]))
                  for i in range(len(meshes)) for q in range(w["P"]))
        ops32 = b32.operators.astype(np.float64)
        lp[name] = {"form": {bem.FORM_DIRECT: "direct", bem.FORM_EXPAND: "expand"}[b32.form],
                    "operators_generated": int(ops32.max()), "col_tile": b32.col_tile,
                    "value": units / wall32, "seconds": wall32, "persistent_kernel_ms": k32,
                    "achieved_tflops": float(np.sum(8.0 * ops32 * sizes ** 2 * w["m"])) / (k32 * 1e-3) / 1e12,
                    "fp32_matrix_peak_tflops": 157.3, "max_rel_err_vs_fp64": err,
                    "speedup_vs_fp64_batch": wall / wall32}
        b32.close()
    res = {
        "workload": w["name"],
        "meshes": f"{w['count']} ellipsoids, geodesic frequency U{{{w['freq'][0]}..{w['freq'][1]}}}, "
                  f"n = {int(sizes.min())}..{int(sizes.max())} (total {int(sizes.sum())}), semi-axes U[0.5, 1.5]",
        "contours": f"|z - c_i| = {w['radius']}, c_i ~ U[3, 7], N = {w['N']}", "m": w["m"], "moments": w["P"],
        "form": {bem.FORM_DIRECT: "direct", bem.FORM_EXPAND: "expand"}[batch.form],
        "operators_generated": [int(x) for x in batch.operators], "col_tile": batch.col_tile,
        "value": units / wall, "unit": "kernel-entry*RHS/s", "seconds": wall,
        "persistent_kernel_ms": kms, "setup_seconds_incl_autotune": setup, "folded": folded,
        "contracted_tflops": achieved, "fp64_mfma_peak_tflops": PEAK_FP64_MFMA_TFLOPS,
        "contracted_frac": achieved / PEAK_FP64_MFMA_TFLOPS,
        "generated_entry_rhs_per_s": float(np.sum(L * sizes ** 2 * w["m"])) / (kms * 1e-3),
        "per_mesh_calls": {"seconds": wall_seq, "value": units / wall_seq},
        "speedup_vs_per_mesh_calls": wall_seq / wall,
        "graph_replay": {"ms": graph_ms, "value": units / (graph_ms * 1e-3),
                         "speedup_vs_per_mesh_calls": wall_seq / (graph_ms * 1e-3),
                         "bitwise_equal_to_eager": graph_equal},
        "max_rel_diff_vs_per_mesh_calls": diff,
        "reduced_precision": lp,
    }
    batch.close()
    for mm in meshes:
        mm.close()
    return res


def large_eigen(level):
    """Eigen-extraction at large n (opt-in, --large-eigen L): the unit icosphere of level L
    (n = 20 4^L; L = 6 is the sweep's n = 81920), circle |z - 5| = 2, N = 64 nodes, 32 probes
    (seed 2), q = 10, tol 1e-12; the Schur complement generated densely on the device and
    factorised there in place by the library's LU.  Reports the eigenvalues with their
    relative residuals, the outer iterations, the times of the assembly, of the
    factorisation and of the whole solve, and the distance of each eigenvalue to the nearest
    interior Dirichlet eigenvalue of the unit sphere (the discretisation error)."""
    import numpy as np
    import torch

    import paper_1906_03938_amd as bem
    import synth
    from paper_1906_03938_amd.eig import ContourSolver

    phase = {"inverse_iteration": 0.0, "rayleigh_ritz": 0.0, "residuals": 0.0}

    class Progress(ContourSolver):
        def _timed(self, name, f, *a):
            t = time.perf_counter()
            out = f(*a)
            phase[name] += time.perf_counter() - t
            return out

        def inverse_iteration(self, u0, lam=None):
            return self._timed("inverse_iteration", super().inverse_iteration, u0, lam)

        def rayleigh_ritz(self, U):
            return self._timed("rayleigh_ritz", super().rayleigh_ritz, U)

        def residuals(self, lam, X):
            res = self._timed("residuals", super().residuals, lam, X)
            print(f"large_eigen: outer iteration {len(self.history) + 1}, {lam.size} Ritz values inside, "
                  f"max residual {res.max() if res.size else float('nan'):.2e}, {time.perf_counter() - t0:.0f} s "
                  f"({', '.join(f'{k} {v:.0f} s' for k, v in phase.items())})", file=sys.stderr, flush=True)
            return res

    xyz, tri = synth.icosphere(level)
    n = tri.shape[0]
    tab = np.loadtxt(os.path.join(ROOT, "tests", "golden", "sphere_dirichlet_eigs.txt"))
    t0 = time.perf_counter()
    with bem.Mesh(xyz, tri) as mesh:
        solver = Progress(mesh, 5.0, 2.0, 64, q=10, tol=1e-12, max_outer=40, lu="device")
        mesh.set_timing(True)
        solver.schur_lu()
        torch.cuda.synchronize()
        t_asm = mesh.last_kernel_ms() * 1e-3
        t_lu = time.perf_counter() - t0
        print(f"large_eigen: n = {n}, assembly {t_asm:.2f} s, assembly + LU {t_lu:.1f} s", file=sys.stderr, flush=True)
        lam, X, res, outer = solver.solve(synth.probe_block(n, 32, seed=2))
        torch.cuda.synchronize()
    total = time.perf_counter() - t0
    dist = [float(np.min(np.abs(l - tab[:, 0]))) for l in lam]
    return {"workload": f"unit icosphere level {level}, n={n}", "contour": "|z - 5| = 2, N = 64", "m": 32,
            "eigenvalues": [[float(l.real), float(l.imag)] for l in lam], "count": int(lam.size),
            "max_rel_residual": float(res.max()) if res.size else None, "outer_iterations": int(outer),
            "assembly_seconds": t_asm, "assembly_plus_device_lu_seconds": t_lu, "total_seconds": total,
            "phase_seconds": phase, "max_distance_to_sphere_eigenvalue": max(dist) if dist else None}


def learned_near_field(freq=158, train_count=2_000_000, steps=40000):
    """The learned near-field correction on the harmonic sphere of 20 freq^2 triangles (seed 5;
    n = 499,280 at freq 158), contour |z - 5| = 1.5, N = 32 nodes, P = 2 moments, m = 64 probes
    (seed 5), near pairs within 2 longest edges.  Trains the network on the GPU with the
    training driver's defaults (2 M seeded samples labelled by the library's quadrature,
    100 k for validation, 40,000 Adam steps of 2048, trust bound 0.2), then times, on the mesh, the folded moment sweep
    once and the correction with the quadrature (series form, and per node) and with the
    network (median of 3), and
    compares the corrected moments: |M_net - M_quad| / |M_quad| per moment (the quadrature
    is the reference), beside the uncorrected moments' distance from the same reference."""
    import numpy as np
    import torch

    import paper_1906_03938_amd as bem
    import synth
    from paper_1906_03938_amd import nfnet

    t0 = time.perf_counter()
    net = nfnet.train(train_count=train_count, val_count=100_000, seed=31, steps=steps, batch=2048)
    t_train = time.perf_counter() - t0
    xyz, tri = synth.harmonic_sphere(freq, seed=5)
    n = len(tri)
    z, w, W = bem.contour_nodes(5.0, 1.5, 32, P=2)
    V = torch.from_numpy(synth.probe_block(n, 64, seed=5)).to("cuda")
    res = {"workload": f"harmonic sphere f={freq}, n={n}", "contour": "|z - 5| = 1.5, N = 32, P = 2", "m": 64,
           "train_samples": train_count, "train_steps": steps, "train_seconds": t_train,
           "train_loss_first_last": [net.history[0][1], net.history[-1][1]],
           "bins_trusted": net.bin_trusted, "bin_validation_error": net.bin_error}
    with bem.Mesh(xyz, tri) as mesh:
        mesh.set_nearfield(2.0)
        res["pairs"] = int(mesh.nearfield_list()[1].size)
        mesh.set_timing(True)
        M = mesh.contour_moments(z, W, V)  # once: about 40 s of kernel time at n = 499,280
        res["sweep_ms"] = mesh.last_kernel_ms()
        res["sweep_form"] = {bem.FORM_DIRECT: "direct", bem.FORM_EXPAND: "expand"}.get(mesh.last_form()[0], "other")
        mesh.set_timing(False)
        Mq = torch.zeros_like(M)
        Mn = torch.zeros_like(M)

        def timed(f, out):
            f(out)
            ms = []
            for _ in range(3):
                out.zero_()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                f(out)
                e1.record()
                e1.synchronize()
                ms.append(e0.elapsed_time(e1))
            return float(np.median(ms))

        model = net.c_model()
        # the quadrature in its default series form (the reference) and per node
        res["quadrature_ms"] = timed(lambda o: mesh.nearfield_moments(z, W, V, out=o), Mq)
        res["quadrature_series_terms"] = mesh.nearfield_last_terms()
        mesh.set_nearfield_mode(bem.NF_NODES)
        res["quadrature_per_node_ms"] = timed(lambda o: mesh.nearfield_moments(z, W, V, out=o), torch.zeros_like(M))
        mesh.set_nearfield_mode(bem.NF_AUTO)
        res["network_ms"] = timed(lambda o: mesh.nearfield_moments_net(model, z, W, V, out=o), Mn)
        _, fb = mesh.nearfield_moments_net(model, z, W, V, out=torch.zeros_like(M), count_fallback=True)
        res["fallback_pairs"] = int(fb)
        res["network_speedup"] = res["quadrature_ms"] / res["network_ms"]
        res["network_speedup_vs_per_node_quadrature"] = res["quadrature_per_node_ms"] / res["network_ms"]
        # the network frozen at the contour centre (one evaluation per pair), freeze_tol 1e-2
        fmodel = net.frozen(1e-2).c_model()
        Mfz = torch.zeros_like(M)
        res["frozen_ms"] = timed(lambda o: mesh.nearfield_moments_net(fmodel, z, W, V, out=o), Mfz)
        _, fbf = mesh.nearfield_moments_net(fmodel, z, W, V, out=torch.zeros_like(M), count_fallback=True)
        res["frozen_fallback_pairs"] = int(fbf)
        res["frozen_speedup"] = res["quadrature_ms"] / res["frozen_ms"]
        res["frozen_speedup_vs_per_node_quadrature"] = res["quadrature_per_node_ms"] / res["frozen_ms"]
        res["moment_error_frozen_vs_quadrature"] = [
            float(torch.linalg.vector_norm((M + Mfz)[p] - (M + Mq)[p]) / torch.linalg.vector_norm((M + Mq)[p]))
            for p in range(2)]
        full_q, full_n, none = M + Mq, M + Mn, M
        res["moment_error_network_vs_quadrature"] = [
            float(torch.linalg.vector_norm(full_n[p] - full_q[p]) / torch.linalg.vector_norm(full_q[p])) for p in range(2)]
        res["moment_error_uncorrected_vs_quadrature"] = [
            float(torch.linalg.vector_norm(none[p] - full_q[p]) / torch.linalg.vector_norm(full_q[p])) for p in range(2)]
        res["correction_error_network"] = [
            float(torch.linalg.vector_norm(Mn[p] - Mq[p]) / torch.linalg.vector_norm(Mq[p])) for p in range(2)]
    print(f"bench: learned near field: quadrature {res['quadrature_ms']:.1f} ms, network {res['network_ms']:.1f} ms",
          file=sys.stderr, flush=True)
    return res


def dense_lu(n=32768, m=64):
    """The inverse iteration's dense LU (bem_lu_factor, bem_lu_solve) on a seeded n x n complex
    Gaussian matrix (torch's Philox generator, seed 1): factorisation time and rate counted as
    8/3 n^3 real flops (the complex LU's flops; the GEMM issues 3/4 of them as MFMA work),
    one solve with m right-hand sides and its relative residual, and the ROCm solver library's
    factorisation of the same matrix (torch.linalg.lu_factor; it takes 32-bit sizes, so only
    for n^2 < 2^31) for comparison."""
    import torch

    from paper_1906_03938_amd import _lib

    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    A0 = torch.complex(torch.randn((n, n), dtype=torch.float64, device="cuda", generator=g),
                       torch.randn((n, n), dtype=torch.float64, device="cuda", generator=g))
    B = torch.complex(torch.randn((n, m), dtype=torch.float64, device="cuda", generator=g),
                      torch.randn((n, m), dtype=torch.float64, device="cuda", generator=g))
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    A = A0.clone()
    torch.cuda.synchronize()
    e0.record()
    lu = _lib.LU(A)
    e1.record()
    X = lu.solve(B)
    e2.record()
    torch.cuda.synchronize()
    t_f, t_s = e0.elapsed_time(e1) * 1e-3, e1.elapsed_time(e2)
    res = (torch.linalg.matrix_norm(A0 @ X - B) / (torch.linalg.matrix_norm(A0) * torch.linalg.matrix_norm(X))).item()
    flops = 8.0 / 3.0 * n ** 3
    out = {"n": n, "matrix": "complex Gaussian, torch Philox seed 1", "info": lu.info, "factor_seconds": t_f,
           "factor_tflops": flops / t_f / 1e12, "flop_count": "8/3 n^3", "fp64_mfma_peak_tflops": 78.6,
           "frac_of_peak": flops / t_f / 1e12 / 78.6, "mfma_issued_frac": 0.75 * flops / t_f / 1e12 / 78.6,
           "solve_m": m, "solve_ms": t_s, "solve_rel_residual": res}
    del lu, X
    print(f"bench: dense LU n = {n}: {t_f:.2f} s", file=sys.stderr, flush=True)
    if n * n < 2 ** 31:
        A.copy_(A0)
        piv = torch.empty(n, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        e0.record()
        torch.linalg.lu_factor(A, out=(A, piv))
        e1.record()
        torch.cuda.synchronize()
        t_r = e0.elapsed_time(e1) * 1e-3
        out["rocsolver_factor_seconds"] = t_r
        out["speedup_vs_rocsolver"] = t_r / t_f
    del A, A0, B
    torch.cuda.empty_cache()
    return out


def near_field(mesh, U, z, W, sweep_kernel_ms, eta=2.0, freq=158):
    """Near-field correction (bem_nearfield_moments, eta = 2): on the headline mesh beside the
    per-node sweep it corrects, and on the harmonic sphere of 20 freq^2 triangles
    (radius 1 + 0.1 sum_{l<=6} c_lm Y_lm, seed 5) with the same nodes, weights and m."""
    import numpy as np
    import torch

    import paper_1906_03938_amd as bem
    import synth

    def timed(msh, V, mode, reps=3):
        """Median ms of the correction alone (zero start) in the given mode, its result and
        the series length it used."""
        msh.set_nearfield_mode(mode)
        out = torch.zeros((W.shape[1], msh.n, V.shape[1]), dtype=torch.complex128, device="cuda")
        msh.nearfield_moments(z, W, V, out=out)  # warm-up, and the correction itself
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            msh.nearfield_moments(z, W, V, out=out)
            e1.record()
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        bem.stream_status()
        terms = msh.nearfield_last_terms()
        out.zero_()
        msh.nearfield_moments(z, W, V, out=out)
        msh.set_nearfield_mode(bem.NF_AUTO)
        return float(np.median(ms)), out, terms

    def both(msh, V, key):
        """Series form (the default) and per-node form: times, and their largest difference
        per weight set on the error scale of either form, sum_j |W[j, p]| |dT(z_j)| V, taken
        as the order-0 set's correction norm times the ratio of the weight sums (the order-1
        set cancels to about 1e-5 of it, so its own norm is not the scale)."""
        ms_s, out_s, terms = timed(msh, V, bem.NF_AUTO)
        ms_n, out_n, _ = timed(msh, V, bem.NF_NODES)
        base = float(torch.linalg.vector_norm(out_n[0]))
        aw = np.abs(W).sum(axis=0)
        diff = max(float(torch.linalg.vector_norm(out_s[p] - out_n[p])) / (base * aw[p] / aw[0])
                   for p in range(out_s.shape[0]))
        del out_s, out_n
        return {f"{key}_ms": ms_s, f"{key}_series_terms": terms, f"{key}_per_node_ms": ms_n,
                f"{key}_series_speedup": ms_n / ms_s, f"{key}_series_vs_per_node_rel_diff": diff}

    res = {"eta": eta, "nodes": len(z), "weight_sets": int(W.shape[1]), "m": int(U.shape[1])}
    t0 = time.perf_counter()
    mesh.set_nearfield(eta)
    res["headline_list_s"] = time.perf_counter() - t0
    res["headline_pairs"] = int(mesh.nearfield_list()[1].size)
    res.update(both(mesh, U, "headline"))
    res["headline_fraction_of_sweep_kernel"] = res["headline_ms"] / sweep_kernel_ms if sweep_kernel_ms else None
    mesh.set_nearfield(0.0)
    xyz, tri = synth.harmonic_sphere(freq, seed=5)
    n = len(tri)
    V = torch.from_numpy(synth.probe_block(n, U.shape[1], seed=5)).to("cuda")
    with bem.Mesh(xyz, tri) as big:
        t0 = time.perf_counter()
        big.set_nearfield(eta)
        res["harmonic_list_s"] = time.perf_counter() - t0
        pairs = int(big.nearfield_list()[1].size)
        res.update(both(big, V, "harmonic"))
    res.update({"harmonic_mesh": f"harmonic sphere f={freq}, n={n}", "harmonic_pairs": pairs,
                "pair_node_evaluations_per_s": pairs * len(z) / (res["harmonic_ms"] * 1e-3),
                "pair_node_evaluations_per_s_per_node_form": pairs * len(z) / (res["harmonic_per_node_ms"] * 1e-3)})
    del V
    torch.cuda.empty_cache()
    return res


def near_field_section():
    """The near-field section on its own: the headline mesh, nodes, weights and probes without
    the sweep (its fraction of the sweep kernel is then not reported)."""
    import torch

    import paper_1906_03938_amd as bem
    import synth

    w = WORKLOAD
    xyz, tri = synth.icosphere(w["level"])
    U = torch.from_numpy(synth.probe_block(tri.shape[0], w["m"], seed=w["seed"])).to("cuda")
    z, _, W = bem.contour_nodes(w["c"], w["radius"], w["N"], P=w["P"])
    with bem.Mesh(xyz, tri) as mesh:
        return near_field(mesh, U, z, W, None)


def eigen_check():
    """Eigenvalues of the sphere-1280 workload (icosphere level 3, |z - 4| < 1.5, N = 32,
    16 probes, seed 1) by the host driver on device sweeps, against the oracle's values
    stored in tests/golden/sphere1280_eigs.txt (written by an oracle-only script)."""
    import numpy as np

    import paper_1906_03938_amd as bem
    import synth
    from paper_1906_03938_amd.eig import eigs_in_contour

    ref = np.loadtxt(os.path.join(ROOT, "tests", "golden", "sphere1280_eigs.txt"))
    lam_ref = np.sort_complex(ref[:, 0] + 1j * ref[:, 1])
    xyz, tri = synth.icosphere(3)
    t0 = time.perf_counter()
    with bem.Mesh(xyz, tri) as mesh:
        lam, _, res, outer = eigs_in_contour(mesh, 4.0, 1.5, 32, synth.probe_block(1280, 16, seed=1))
    dt = time.perf_counter() - t0
    ok = lam.size == lam_ref.size
    err = float(np.max(np.abs(np.sort_complex(lam) - lam_ref) / np.abs(lam_ref))) if ok else None
    return {"workload": "sphere-1280", "eigenvalues": [[float(l.real), float(l.imag)] for l in np.sort_complex(lam)],
            "max_rel_err_vs_oracle": err, "max_rel_residual": float(res.max()), "outer_iterations": int(outer),
            "seconds": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-eigen-check", action="store_true")
    ap.add_argument("--no-precision-form", action="store_true")
    ap.add_argument("--no-batched-form", action="store_true")
    ap.add_argument("--no-near-field", action="store_true")
    ap.add_argument("--no-dense-lu", action="store_true")
    ap.add_argument("--no-learned-near-field", action="store_true")
    ap.add_argument("--dense-lu-only", type=int, default=0, metavar="N",
                    help="only run the dense LU section at size N and print its JSON")
    ap.add_argument("--only", default="", metavar="SECTIONS",
                    help="only run the named sections (comma-separated: precision_form, precision_sweeps, "
                         "batched_form, near_field, learned_near_field, dense_lu, eigen_check) and print their JSON")
    ap.add_argument("--large-eigen", type=int, default=0, metavar="L",
                    help="also run the eigen-extraction on the unit icosphere of level L (n = 20 4^L; "
                         "L = 6: n = 81920, about 8 minutes) with the library's LU")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (3 times), the "
                         "reference kernel for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sweep's multi-GPU "
              "row split is a design note, not built.", file=sys.stderr)
        sys.exit(2)
    if args.dense_lu_only:
        print(json.dumps({"dense_lu": dense_lu(args.dense_lu_only)}), flush=True)
        return
    if args.only:
        sections = {"precision_form": precision_form, "precision_sweeps": precision_sweeps,
                    "batched_form": batched_form, "near_field": near_field_section,
                    "learned_near_field": learned_near_field, "dense_lu": dense_lu, "eigen_check": eigen_check}
        res = {}
        for name in args.only.split(","):
            if name not in sections:
                print(f"unknown section {name!r}; known: {', '.join(sections)}", file=sys.stderr)
                sys.exit(2)
            res[name] = sections[name]()
            print(f"bench: {name} done", file=sys.stderr, flush=True)
        print(json.dumps(res), flush=True)
        return

    import numpy as np
    import torch

    import paper_1906_03938_amd as bem
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        nbytes = args.calibrate_copy // 8 * 8
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "dispatches": 3}), flush=True)
        return
    w = WORKLOAD
    xyz, tri = synth.icosphere(w["level"])
    n = tri.shape[0]
    Vh = synth.probe_block(n, w["m"], seed=w["seed"])
    U = torch.from_numpy(Vh).to("cuda")
    mesh = bem.Mesh(xyz, tri)
    mesh.set_timing(True)
    Pout = torch.empty((w["N"], w["m"], w["m"]), dtype=torch.complex128, device="cuda")
    Mout = torch.empty((w["P"], n, w["m"]), dtype=torch.complex128, device="cuda")
    units = w["N"] * n * n * w["m"]
    khash = kernel_source_hash()

    def step(form):
        z, _, W = bem.contour_nodes(w["c"], w["radius"], w["N"], P=w["P"])
        mesh.rr_project(z, U, W=W, out=Pout, moments_out=Mout, form=form)
        return z

    def run(form, steps, warmup):
        """warm-up steps, then `steps` timed ones: wall clock over all of them (bracketed by
        device synchronisations), HIP events around each step on the call's stream (torch's
        current stream) and the library's events around each sweep kernel."""
        for _ in range(warmup):
            step(form)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        kernel_ms = []
        t0 = time.perf_counter()
        for e0, e1 in ev:
            e0.record()
            z = step(form)
            e1.record()
            kernel_ms.append(mesh.last_kernel_ms())  # waits for this step's sweep kernel only
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        bem.stream_status()
        step_ms = [e0.elapsed_time(e1) for e0, e1 in ev]
        used, L = mesh.last_form()
        return z, elapsed, step_ms, kernel_ms, used, L

    def roofline(L, kernel_ms, traffic_file):
        flops = 8.0 * L * n * n * w["m"]  # 8 real flops per complex multiply-add of each contracted operator
        kms = float(np.mean(kernel_ms))
        achieved = flops / (kms * 1e-3) / 1e12
        return {
            "bound": "mfma",
            "achieved": achieved,
            "peak": PEAK_FP64_MFMA_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_MFMA_TFLOPS,
            "traffic": load_traffic(traffic_file, khash),
            "kernel": "sweep_kernel",
            "kernel_ms": kms,
            "kernel_ms_median": float(np.median(kernel_ms)),
            "flops_per_launch": flops,
            # the kernel forms each complex product with three real multiplications (Gauss):
            # the matrix cores execute 6 of the 8 flops counted above
            "mfma_issued_frac": 0.75 * achieved / PEAK_FP64_MFMA_TFLOPS,
            "kernel_hash": khash,
        }

    def progress(msg):
        print(f"bench: {msg}", file=sys.stderr, flush=True)

    # the headline: the per-node sweep
    z, elapsed, step_ms, kernel_ms, used_form, L = run(bem.FORM_DIRECT, args.steps, args.warmup)
    progress(f"per-node sweep {1e3 * elapsed / args.steps:.0f} ms per step")
    assert used_form == bem.FORM_DIRECT and L == w["N"]
    ms_per_step = 1e3 * elapsed / args.steps
    out = {
        "metric": "kernel-entry*RHS/s of sum_j T(z_j)V sweep (rr_project + fused moments, per-node form)",
        "value": units / (elapsed / args.steps),
        "unit": "kernel-entry*RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "step_ms_median_events": float(np.median(step_ms)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": w["name"],
            "mesh": f"unit icosphere level {w['level']}, n={n} triangles",
            "contour": f"circle c={w['c']} r={w['radius']}, N={w['N']} trapezoidal nodes",
            "m": w["m"], "moments": w["P"], "seed": w["seed"],
            "form": "direct",
            "operators_generated": L,
        },
        "roofline": roofline(L, kernel_ms, "sweep_direct_sphere81920_traffic.json"),
    }
    # the Taylor-expansion form of the same call (what FORM_AUTO takes here)
    reps = max(3, min(args.steps, 5))
    _, el_t, step_t, kms_t, used_t, L_t = run(bem.FORM_AUTO, reps, 1)
    t_step = el_t / reps
    progress(f"Taylor form {1e3 * t_step:.0f} ms per step")
    out["taylor_form"] = {
        "call": "rr_project with 2 fused moments, FORM_AUTO (Taylor expansion about the contour centre)",
        "form": "expand" if used_t == bem.FORM_EXPAND else "direct",
        "operators_generated": L_t,
        "steps": reps,
        "ms_per_step": 1e3 * t_step,
        "step_ms_median_events": float(np.median(step_t)),
        "effective_value": units / t_step,
        "effective_unit": "kernel-entry*RHS/s counted as N n^2 m (N = 64 nodes) although L n^2 m are contracted",
        "contracted_value": L_t * n * n * w["m"] / t_step,
        "contracted_unit": "contracted operator entry*RHS/s (L n^2 m)",
        "speedup_vs_per_node_step": ms_per_step / (1e3 * t_step),
        "roofline": roofline(L_t, kms_t, "sweep_sphere81920_traffic.json"),
    }
    # the folded form: contour_moments with P = 2 weight sets generates every operator of each
    # entry but contracts only the two folds (reported beside, not as, the per-node sweep)
    form = bem.FORM_AUTO
    z2, _, W2 = bem.contour_nodes(w["c"], w["radius"], w["N"], P=w["P"])
    mesh.contour_moments(z2, W2, U, out=Mout, form=form)
    fold_ms = []
    for _ in range(2):
        mesh.contour_moments(z2, W2, U, out=Mout, form=form)
        fold_ms.append(mesh.last_kernel_ms())
    kms = out["roofline"]["kernel_ms"]
    out["folded_moments"] = {
        "call": f"contour_moments, P = {w['P']} weight sets on the headline mesh, nodes and probes",
        "kernel_ms": float(np.mean(fold_ms)), "value": units / (float(np.mean(fold_ms)) * 1e-3),
        "unit": "kernel-entry*RHS/s (effective: N n^2 m)", "contractions": w["P"],
        "operators_generated": mesh.last_form()[1],
        "speedup_vs_per_node_sweep_kernel": kms / float(np.mean(fold_ms)),
    }
    if not args.no_near_field:
        out["near_field"] = near_field(mesh, U, z2, W2, kms)
        progress("near field done")
    mesh.close()
    if not args.no_eigen_check:
        out["eigen_check"] = eigen_check()
        progress("eigen check done")
    if not args.no_precision_form:
        out["precision_form"] = precision_form()
        progress("precision form done")
    if not args.no_batched_form:
        out["batched_form"] = batched_form()
        progress("batched form done")
    if not args.no_learned_near_field:
        out["learned_near_field"] = learned_near_field()
        progress("learned near field done")
    if not args.no_dense_lu:
        out["dense_lu"] = dense_lu()
        progress("dense LU done")
    if args.large_eigen:
        out["large_eigen"] = large_eigen(args.large_eigen)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(xyz, tri, z, Vh)
        progress("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
