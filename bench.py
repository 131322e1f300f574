"""Benchmark: space-time DoF/s of the fast-diagonalization solve on one MI355X.

One step is the whole hot path for one right-hand side: host temporal
eigen-step, band fill and batched LDL^T of all spatial blocks (fdm_factor),
then fdm_solve (rhs transform, sweeps, back-transform, FP64 Kronecker residual
and refinement until ||F - K Psi|| / ||F|| <= 1e-10).  Matrix assembly and
the load vector are excluded, as in the paper's timings (Sec. 4).

Workload: unit square, n = 256 cells per side (n_x = 65025), 256 uniform P1
time elements on (0, 2) (n_t = 256, 16,646,400 space-time dofs), manufactured
psi = sin(pi x) sin(pi y)(1 + t^2) e^{4 pi i t} homogenised by psi_0.  The
headline runs FP32 factors and sweeps with FP64 refinement; the same steps
with FP64 factors give the speedup.

Prints one JSON line.  `--gpus N` with N > 1 is not supported (one GPU).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MFMA_PEAK_TFLOPS = {32: 157.3, 64: 78.6}     # MI355X dense matrix peaks (FP32, FP64)
HBM_PEAK_GBS = 8000.0


def ldlt_flops(n_x, kd):
    """Algorithmic real flops of one banded L D L^T: column j updates the
    t_j (t_j + 1)/2 lower-triangle entries of its trailing window with one
    complex multiply-add each (8 real flops), t_j = min(kd, n_x - 1 - j)."""
    import numpy as np
    t = np.minimum(kd, n_x - 1 - np.arange(n_x)).astype(np.float64)
    return float(8.0 * np.sum(t * (t + 1) / 2))


def kernel_source_hash():
    p = os.path.join(ROOT, "paper_2504_07269_amd", "csrc", "kernels.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def measured_traffic(precision, kernel="ldlt"):
    """HBM bytes per launch of k_ldlt (or k_sweep) from the committed rocprofv3
    counter runs, if they were taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "%s_c2_fp%d_traffic.json" % (kernel, precision))
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernels_hip_sha256_16") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def sweep_roofline(reps, n_x, kd, n_t):
    """HBM roofline of the FP32 sweep (one forward + backward pass over every
    block, one rhs): algorithmic bytes = the factor slab once per direction,
    g and u read once and u written twice (complex128); time per launch = the
    sweep time of a step over its launches (one per application of the
    inverse)."""
    slab = n_t * n_x * (kd + 1) * 8
    alg = 2 * slab + 4 * n_t * n_x * 16
    launches = sum(r["iterations"] + 1 for r in reps)
    ms = sum(r["ms_sweeps"] for r in reps) / launches
    achieved = alg / (ms / 1000.0) / 1e9
    return {"kernel": "k_sweep (FP32)", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(32, "sweep"), "bytes_per_launch": alg,
            "ms_per_launch": ms}


def progress(msg):
    sys.stderr.write("[bench] %s\n" % msg)
    sys.stderr.flush()


def run_steps(st, torch, inputs, precision, steps, warmup, tol, max_iter, refine):
    Mt, Bt, Ms, As, n, F = inputs
    reports = []

    def one():
        h = st.fdm_factor(Mt, Bt, Ms, As, n, precision=precision, tol=tol, max_iter=max_iter, refine=refine)
        Psi = h.solve(F)
        rep = dict(h.last_report)
        h.close()
        return Psi, rep

    for i in range(warmup):
        _, rep = one()
        progress("fp%d warmup %d: %.1f ms, ldlt %.1f ms, %d extra applications of the inverse, residual %.2e"
                 % (precision, i, rep["ms_total"] + rep["ms_eig"] + rep["ms_factor"], rep["ms_ldlt"],
                    rep["iterations"], rep["rel_residual"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        Psi, rep = one()
        reports.append(rep)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    progress("fp%d: %d timed steps, %.1f ms per step" % (precision, steps, (t1 - t0) * 1000.0 / steps))
    return (t1 - t0) * 1000.0 / steps, reports, Psi


def reuse_rates(st, torch, inputs, precision, steps, tol, max_iter, refine):
    """Solve-only and adjoint rates with the factors reused: one fdm_factor,
    then `steps` forward and `steps` adjoint solves (refinement included), each
    after one untimed call."""
    Mt, Bt, Ms, As, n, F = inputs
    h = st.fdm_factor(Mt, Bt, Ms, As, n, precision=precision, tol=tol, max_iter=max_iter, refine=refine)
    out = {}
    try:
        for name, fn in (("solve", h.solve), ("adjoint", h.solve_adjoint)):
            fn(F)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps = []
            for _ in range(steps):
                fn(F)
                reps.append(dict(h.last_report))
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1000.0 / steps
            out[name] = {"ms": ms, "iterations": [r["iterations"] for r in reps],
                         "rel_residual": [r["rel_residual"] for r in reps]}
            progress("fp%d %s only: %.1f ms, %d extra applications of the inverse"
                     % (precision, name, ms, reps[-1]["iterations"]))
    finally:
        h.close()
    return out


def cpu_baseline(wl, Mt, Bt, F_np, stride):
    from oracle import baseline
    _, t = baseline.fdm_timed(Mt, Bt, wl.n, F_np, block_stride=stride)
    return {"value": wl.dofs / t["total"], "unit": "dof/s", "cores": t["workers"], "kind": "oracle",
            "sample": "paper-form FDM (numpy eig + GEMMs, scipy splu per block in %d worker processes); "
                      "%d of %d spatial blocks solved, their wall time scaled by %d/%d; eigen-step and "
                      "transforms complete" % (t["workers"], t["blocks_solved"], t["blocks_total"],
                                               t["blocks_total"], t["blocks_solved"]),
            "seconds": {k: round(v, 3) for k, v in t.items() if isinstance(v, float)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--max-iter", type=int, default=60)
    ap.add_argument("--refine", default="gmres", choices=["gmres", "plain", "block"],
                    help="refinement of the FP32 solve (the FP64 comparison always uses gmres)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-block-stride", type=int, default=2)
    ap.add_argument("--factor-only", type=int, default=0, metavar="PRECISION",
                    help="profiling aid: run one fdm_factor of the workload in this precision and exit")
    ap.add_argument("--copy-probe", type=float, default=0.0, metavar="GIB",
                    help="profiling aid: one device-to-device copy of this many GiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only; --gpus %d is not supported (the solver is a single-GPU "
              "library; multi-GPU sharding by time blocks is a design note, not built)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2504_07269_amd as st
    import synth

    if args.copy_probe > 0:
        nbytes = int(args.copy_probe * 2 ** 30)
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        progress("copied %d bytes" % nbytes)
        return

    wl = synth.WORKLOADS[args.workload]
    if wl.p_t != 1 and wl.n > 256:
        print("workload %s does not fit one GPU unchunked" % wl.name, file=sys.stderr)
        sys.exit(2)
    nodes = synth.uniform_nodes(wl.T, wl.N_t)
    Mt, Bt, _, _ = st.assemble_1d_time(nodes, wl.p_t)
    Ms, As, n_x, kd = st.assemble_2d_space(wl.n)
    F_np = synth.manufactured_rhs(wl)
    F = torch.from_numpy(F_np).to("cuda:0")
    inputs = (Mt, Bt, Ms, As, wl.n, F)
    if args.factor_only:
        h = st.fdm_factor(Mt, Bt, Ms, As, wl.n, precision=args.factor_only, tol=args.tol)
        torch.cuda.synchronize()
        progress("factor only: fp%d done" % args.factor_only)
        h.close()
        return

    ms32, reps32, _ = run_steps(st, torch, inputs, 32, args.steps, args.warmup, args.tol, args.max_iter, args.refine)
    value = wl.dofs / (ms32 / 1000.0)
    avg = lambda reps, k: float(np.mean([r[k] for r in reps]))
    ms_ldlt = avg(reps32, "ms_ldlt")
    flops = ldlt_flops(n_x, kd) * wl.n_t
    achieved = flops / (ms_ldlt / 1000.0) / 1e12
    out = {
        "metric": "space-time DoF/s of FDM solve at 1e-10 rel err; FP32+IR vs FP64 speedup",
        "value": value, "unit": "dof/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms32, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 factors+sweeps, c128 residual/refinement", "data": "synthetic",
        "config": {"workload": "FDM solve, unit square n=%d cells/side (n_x=%d, kd=%d), %d P%d time elements "
                               "on (0,%g) (n_t=%d), %d space-time dofs, 1 rhs, manufactured psi omega=%.4g, "
                               "FP32 LDL^T + FP64 %s refinement to %.0e"
                               % (wl.n, n_x, kd, wl.N_t, wl.p_t, wl.T, wl.n_t, wl.dofs, wl.omega,
                                  {"gmres": "GMRES", "plain": "plain", "block": "block GMRES"}[args.refine],
                                  args.tol),
                   "dofs": wl.dofs, "n_x": n_x, "n_t": wl.n_t, "rhs": 1},
        "roofline": {"kernel": "k_ldlt (FP32)", "bound": "mfma", "achieved": achieved,
                     "peak": MFMA_PEAK_TFLOPS[32], "unit": "TFLOP/s", "frac": achieved / MFMA_PEAK_TFLOPS[32],
                     "traffic": measured_traffic(32), "flops_per_launch": flops, "ms_per_launch": ms_ldlt},
        "roofline_sweep": sweep_roofline(reps32, n_x, kd, wl.n_t),
        "stages_ms_fp32": {k: avg(reps32, k) for k in ("ms_eig", "ms_band_fill", "ms_ldlt", "ms_sweeps",
                                                        "ms_transforms", "ms_residual", "ms_factor", "ms_total")},
        "refinement_fp32": {"method": args.refine, "iterations": [r["iterations"] for r in reps32],
                            "rel_residual": [r["rel_residual"] for r in reps32],
                            "history": reps32[-1]["history"]},
        "kappa_x": reps32[-1]["kappa_x"],
    }
    reuse = reuse_rates(st, torch, inputs, 32, args.steps, args.tol, args.max_iter, args.refine)
    out["reused_factors_fp32"] = {name: dict(r, dof_per_s=wl.dofs / (r["ms"] / 1000.0)) for name, r in reuse.items()}
    if not args.no_fp64:
        ms64, reps64, _ = run_steps(st, torch, inputs, 64, args.steps, args.warmup, args.tol, args.max_iter, "gmres")
        v64 = wl.dofs / (ms64 / 1000.0)
        out["fp64"] = {"value": v64, "ms_per_step": ms64,
                       "stages_ms": {k: avg(reps64, k) for k in ("ms_eig", "ms_band_fill", "ms_ldlt", "ms_sweeps",
                                                                 "ms_transforms", "ms_residual", "ms_total")},
                       "iterations": [r["iterations"] for r in reps64],
                       "rel_residual": [r["rel_residual"] for r in reps64],
                       "ldlt_tflops": ldlt_flops(n_x, kd) * wl.n_t / (avg(reps64, "ms_ldlt") / 1000) / 1e12}
        out["speedup_fp32ir_vs_fp64"] = value / v64
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle FDM on the host cores)")
        out["cpu_baseline"] = cpu_baseline(wl, Mt, Bt, F_np, args.cpu_block_stride)
        progress("cpu baseline: %.3g dof/s" % out["cpu_baseline"]["value"])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
