"""Benchmark: frequency solves per second of the exponential-window BEM.

One step is the whole transient solve of the pressurised spherical cavity
at 61,440 unknowns (icosphere level 5, 20,480 triangles): for each of the
65 damped frequencies s_k (N_f = 128) the H-matrix operator (leaf 64,
eta = 1, ACA 1e-5), the right-hand side and the block-diagonal
preconditioner are assembled, the initial guess is extrapolated from the
three previous solutions, GMRES runs to a 1e-6 relative residual; then the
windowed, de-damped inverse transform gives the time response.  Inputs are
resident on the GPU before the timed region.

The default line also carries, each timed on its own after the main steps:
``quad_variant``, the same transient with the plain quadratic
extrapolation 3 a1 - 3 a2 + a3 as the initial guess; and ``learned_fp32``,
the headline comparison on the same geometry under spherical-harmonic
pressures: held-out loads solved by plain FP64 (complex128 factors,
least-squares extrapolation) and by the learned guess with complex64 far
factors (FP64 Arnoldi and residuals), the guess trained (untimed) on
--learned-train other loads.

Prints one JSON line (rank 0).  Only one GPU is used: --gpus above 1 exits.
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "freq-solves/s at N=61k, 1e-6 resid: learned+FP32 vs plain FP64; H-matvec GB/s"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sub", type=int, default=None, help="icosphere level (default 5)")
    ap.add_argument("--store", choices=["c128", "c64"], default="c128")
    ap.add_argument("--no-pipeline-variant", action="store_true",
                    help="skip timing the pipelined frequency loop (next ACA overlapping GMRES)")
    ap.add_argument("--c64-variant", action="store_true",
                    help="also time the complex64-factor variant")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variant-steps", type=int, default=1,
                    help="cavity workload: transients timed with the plain quadratic extrapolation "
                         "3 a1 - 3 a2 + a3 after the least-squares one (Sec. 4.2, K = 3), on the "
                         "same context (0: skip)")
    ap.add_argument("--learned-train", type=int, default=48,
                    help="cavity workload: training loads of the learned + FP32 comparison "
                         "(spherical-harmonic pressures on the same geometry; 0: skip)")
    ap.add_argument("--learned-held", type=int, default=1,
                    help="cavity workload: held-out loads timed in each leg of that comparison")
    ap.add_argument("--learned-modes", type=int, default=128,
                    help="reduced coordinates of the learned guess")
    ap.add_argument("--aca-reuse", type=int, choices=[0, 1], default=None,
                    help="start each frequency's ACA from the previous pivots (library default if unset)")
    ap.add_argument("--cpu-rows", type=int, default=48)
    ap.add_argument("--workload", choices=["cavity", "rod-table1", "rod-long", "learned", "batch12", "scene", "loads",
                                           "scene-waves"],
                    default="cavity",
                    help="cavity: the frequency-solve benchmark (default); rod-table1: the "
                         "three damping / extrapolation cases of the paper's Table 1 on its "
                         "prismatic rod; rod-long: the rod's long-time run of Sec. 5.1 (N_w = 512, "
                         "257 solves) against the 1-D closed form; learned: the cavity under spherical-harmonic "
                         "pressures, learned guess with complex64 factors against plain FP64; "
                         "batch12: twelve cavities of uneven size (levels 3-5) solved "
                         "concurrently against one at a time; scene: twelve cavities in one "
                         "mesh scattering a plane S-wave (level 3 unless --sub); loads: the "
                         "cavity under --n-loads pressure loads through one frequency loop "
                         "against one transient per load; scene-waves: the scene under --n-loads "
                         "incident S-waves of different directions, the same comparison")
    ap.add_argument("--lockstep", action="store_true",
                    help="batch12 workload: each wave in lock-step over the frequency index, one "
                         "concatenated matvec (a replayed HIP graph) per Arnoldi step for the wave")
    ap.add_argument("--wave", type=int, default=6,
                    help="batch12 workload: problems alive and solved concurrently at once")
    ap.add_argument("--fp64-reference", action="store_true",
                    help="batch12 and scene workloads: also solve every problem with complex128 factors "
                         "(untimed) and report the complex64 results' relative L2 error against them")
    ap.add_argument("--total-field", action="store_true",
                    help="scene workload: the total-field formulation of the incident wave "
                         "(right-hand side u_inc itself, O(N) per frequency; outputs the total "
                         "displacement) instead of the scattered one (O(N^2) sum U t_sc)")
    ap.add_argument("--aca-batch-mb", type=int, default=0,
                    help="scene workload: approximate the far blocks in batches of about this many "
                         "MiB of complex128 work area, converting each to complex64 as it "
                         "finishes (0: all at once)")
    ap.add_argument("--per-frequency", action="store_true",
                    help="scene workload: drive the frequency loop from here (one solve per "
                         "frequency, a progress line each, then the inverse transform) instead "
                         "of one library call per transient; the default at level 5")
    ap.add_argument("--mv-mfma", type=int, choices=[0, 1], default=1,
                    help="loads workload: eight-right-hand-side matvecs on the FP64 matrix cores (1) or the "
                         "vector units (0)")
    ap.add_argument("--n-loads", type=int, default=8,
                    help="loads workload: loads solved through one frequency loop")
    ap.add_argument("--train-cases", type=int, default=8,
                    help="learned workload: loads the guess is trained on")
    ap.add_argument("--rod-div", type=int, default=20,
                    help="rod mesh: cells per unit length (20 -> 11,200 triangles)")
    ap.add_argument("--no-read-probe", action="store_true",
                    help="skip timing a plain streaming read of 8 GiB (torch's sum over float64), the "
                         "practical HBM read rate the matvec's fraction is set against")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 1 GiB device-to-device three times (a kernel of known "
                         "traffic that calibrates the HBM counters)")
    ap.add_argument("--traffic-summary", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "RUN_LOG"),
                    help="no run: summarise two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of "
                         "'bench.py --copy-probe ...' into profiles/hmatvec_traffic.json, with the "
                         "algorithmic bytes from the bench line in the FETCH_SIZE run's output (RUN_LOG)")
    return ap.parse_args()


def _counter_means(d, counter):
    """Mean per dispatch of one counter, per kernel name, from a rocprofv3
    --pmc csv directory (the counter_collection file)."""
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    acc = {}
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") != counter:
                    continue
                k = r["Kernel_Name"]
                key = (k, r.get("Dispatch_Id", r.get("Correlation_Id", "")))
                acc.setdefault(k, {}).setdefault(key, 0.0)
                acc[k][key] += float(r["Counter_Value"])  # summed over the counter's instances
    return {k: list(v.values()) for k, v in acc.items()}


def _run_algorithmic_bytes(log_path):
    """algorithmic_bytes_per_launch of the bench line in a run's log."""
    with open(log_path) as f:
        for line in f:
            line = line.strip()
            if line.startswith("{") and "algorithmic_bytes_per_launch" in line:
                return json.loads(line)["roofline"]["algorithmic_bytes_per_launch"]
    raise SystemExit(f"no bench line with algorithmic_bytes_per_launch in {log_path}")


def traffic_summary(fetch_dir, write_dir, out_path=None, run_log=None):
    """HBM bytes of one single-vector matvec from the FETCH_SIZE and
    WRITE_SIZE runs, each counter scaled by what it reads for the 1 GiB
    device copy of --copy-probe; written with the hash of the matvec source
    it was taken on and, from the counter run's own bench line (run_log),
    the algorithmic bytes of the operator it applied."""
    fe = _counter_means(fetch_dir, "FETCH_SIZE")
    wr = _counter_means(write_dir, "WRITE_SIZE")

    def pick(tab, pred):
        ks = [k for k in tab if pred(k)]
        if not ks:
            raise SystemExit("kernel not found in the counters")
        k = max(ks, key=lambda k: len(tab[k]))  # the shape that ran most often
        return k, sum(tab[k]) / len(tab[k]), len(tab[k])

    def pick_copy(tab):
        # the 1 GiB copies: the largest dispatches of the runtime's copy kernel
        # (it also serves the run's small copies)
        ks = [k for k in tab if "copy" in k.lower()]
        if not ks:
            raise SystemExit("copy kernel not found in the counters")
        k = max(ks, key=lambda k: max(tab[k]))
        big = [v for v in tab[k] if v >= 0.5 * max(tab[k])]
        return k, sum(big) / len(big)

    ck, cf = pick_copy(fe)
    _, cw = pick_copy(wr)
    gib = float(1 << 30)
    fscale, wscale = gib / (cf * 1024.0), gib / (cw * 1024.0)
    out = {"source_sha256_16": _hash(os.path.join(ROOT, "paper_1212_3032_amd", "csrc", "hmatvec.hip")),
           "copy_calibration": {"copy_kernel": ck, "copy_bytes": int(gib), "fetch_KiB_reported": cf,
                                "write_KiB_reported": cw, "fetch_scale": fscale, "write_scale": wscale},
           "kernels": {}}
    total = 0.0
    for name, pred in (("far_vt", lambda k: "k_far_vt<" in k and ", 1, " in k),
                       ("hmv", lambda k: "k_hmv<1>" in k), ("reduce", lambda k: "k_hmv_reduce" in k)):
        k, f, n = pick(fe, pred)
        _, w, _ = pick(wr, pred)
        b = (f * fscale + w * wscale) * 1024.0
        total += b
        out["kernels"][name] = {"kernel": k, "fetch_KiB": f, "write_KiB": w, "dispatches": n, "hbm_bytes": b}
    out["hbm_bytes_per_matvec"] = total
    if run_log:
        out["algorithmic_bytes_per_launch"] = _run_algorithmic_bytes(run_log)
    p = out_path or os.path.join(ROOT, "profiles", "hmatvec_traffic.json")
    with open(p, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))
    return out


def copy_probe():
    import torch
    n = 1 << 30
    a = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def read_probe():
    """GB/s of torch's float64 sum over 8 GiB (best of five, after one warm run)."""
    import torch
    a = torch.ones((8 << 30) // 8, dtype=torch.float64, device="cuda:0")
    a.sum()
    torch.cuda.synchronize()
    best = 1e30
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        a.sum()
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a
    torch.cuda.empty_cache()
    return (8 << 30) / (best * 1e-3) / 1e9


def _hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_from_profiles(bytes_per_launch, path=None):
    """HBM bytes per matvec from the committed rocprofv3 counter summary, if
    it was taken on the current matvec source and on an operator of the same
    algorithmic bytes (within 0.5%; the ranks, hence the bytes, change with
    the approximation), else None."""
    p = path or os.path.join(ROOT, "profiles", "hmatvec_traffic.json")
    src = os.path.join(ROOT, "paper_1212_3032_amd", "csrc", "hmatvec.hip")
    try:
        with open(p) as f:
            t = json.load(f)
        if t.get("source_sha256_16") != _hash(src):
            return None
        alg = t.get("algorithmic_bytes_per_launch")
        if alg is None or not abs(alg - bytes_per_launch) <= 0.005 * bytes_per_launch:
            return None
        return t["hbm_bytes_per_matvec"]
    except (OSError, KeyError, ValueError):
        return None


def run_gpu(args, store, pipeline=0, guess=None, after=None):
    """Time --steps transients of the level-5 cavity on one context after
    --warmup; ``after(ctx, d, u)`` runs on the same (warm) context before it
    is closed and its result is returned as the fifth value."""
    import torch
    from paper_1212_3032_amd import ewbem as E
    from synth import config_inputs

    d = config_inputs(2, sub=args.sub)
    dev = torch.device("cuda:0")
    ctx = E.Context(0)
    E.setup_from_inputs(
        ctx, d,
        op=dict(kind=E.OP_HMAT, leaf_size=64, eta_adm=1.0, aca_tol=1e-5,
                far_store=E.STORE_C64 if store == "c64" else E.STORE_C128,
                aca_batch_mb=args.aca_batch_mb if store == "c64" else 0,
                **({} if args.aca_reuse is None else {"aca_reuse": args.aca_reuse})),
        solver=dict(tol=1e-6, guess=E.GUESS_SEM if guess is None else guess, sem_k=3,
                    precond=E.PREC_LEAF, pipeline=pipeline))
    N = 3 * len(d["tri"])
    n_f = d["n_f"]
    u = torch.zeros(n_f * N, dtype=torch.float64, device=dev)
    for w in range(args.warmup):
        st = ctx.solve_transient(u)
        print(f"# warmup {w}: {st['n_solves']} solves, {st['iters_total']} its, "
              f"{st['t_assemble_ms']:.0f} ms assembly, {st['t_gmres_ms']:.0f} ms gmres",
              file=sys.stderr, flush=True)
    tot = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        st = ctx.solve_transient(u)
        print(f"# step {s}: {st['iters_total']} its, resid_max {st['resid_max']:.2e}",
              file=sys.stderr, flush=True)
        if tot is None:
            tot = dict(st)
        else:
            for k, v in st.items():
                if k in ("resid_max", "iters_max", "rank_max"):
                    tot[k] = max(tot[k], v)
                elif k in ("matvec_bytes", "stored_bytes", "n_near", "n_far", "rank_sum"):
                    tot[k] = v
                else:
                    tot[k] += v
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    info = ctx.info()
    tot["matvec_shapes"] = {"cols_per_wave": info["mv_cols"], "task_div": info["mv_task_div"],
                            "tuned": info["mv_tuned"], "tuned_ms": info["mv_tune_best_ms"],
                            "default_ms": info["mv_tune_default_ms"]}
    tot["u_last"] = u.cpu().numpy()  # the last timed transient (untimed copy)
    free, total = torch.cuda.mem_get_info()
    tot["device_memory_GB"] = (total - free) / 1e9  # the context, torch's buffers and the runtime
    tot["library_memory_GB"] = {"total": info["lib_device_bytes"] / 1e9,  # the context's own buffers
                                "far_work_areas": info["far_work_bytes"] / 1e9,
                                "aca_scratch": info["aca_scratch_bytes"] / 1e9,
                                "near_field": 16.0 * info["near_entries"] / 1e9}
    extra = after(ctx, d, u) if after is not None else None
    ctx.close()
    return d, N, elapsed, tot, extra


def rod_table1(args):
    """Sec. 5.1, Table 1: total GMRES iterations over the first N_w/2 + 1 = 129
    frequencies of the prismatic rod (3 x 1 x 1, nu = 0, fixed end, step
    traction at the free end), tol 1e-5, block-diagonal preconditioner, for
    kappa = 2 without extrapolation, kappa = 4 without, and kappa = 4 with
    the extrapolation (K = 4).  Lengths in metres scaled so that mu = rho = 1;
    the paper's T = 0.0155 s is 26.8 L / c, kept in those units."""
    import torch
    from paper_1212_3032_amd import ewbem as E
    from synth import box_mesh, ramp_history

    L = 3.0
    n = args.rod_div
    xyz, tri, face = box_mesh((L, 1, 1), (3 * n, n, n), origin=(0, -0.5, -0.5))
    bc = (face == 0).astype(np.int32)
    given = np.zeros((len(tri), 3))
    given[face == 1, 0] = -1.0
    c_bar = np.sqrt(2.0)                       # E = 2 mu (nu = 0), rho = 1
    period = 26.79 * L / c_bar
    n_f = 256
    hist = ramp_history(n_f, period, 0.0)
    N = 3 * len(tri)
    cases = [("kappa=2, no SEM", 2.0, E.GUESS_ZERO, 29237, 16.0),
             ("kappa=4, no SEM", 4.0, E.GUESS_ZERO, 21758, 14.4),
             ("kappa=4, SEM K=4", 4.0, E.GUESS_SEM, 17562, 12.1)]
    out = []
    dev = torch.device("cuda:0")
    for name, kappa, guess, paper_its, paper_h in cases:
        ctx = E.Context(0)
        ctx.set_mesh(xyz, tri, exterior=False)
        ctx.set_material(1.0, 1.0, 0.0)
        ctx.set_time(period, n_f, kappa * np.log(10.0) / period, E.WINDOW_HANN)
        ctx.set_load_mixed(bc, given, hist)
        ctx.set_operator(kind=E.OP_HMAT, leaf_size=64, eta_adm=1.0, aca_tol=1e-5)
        ctx.set_solver(tol=1e-5, guess=guess, sem_k=4, precond=E.PREC_LEAF, maxit=2000)
        u = torch.zeros(n_f * N, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ctx.solve_transient(u, allow_noconv=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ctx.close()
        print(f"# {name}: {st['iters_total']} its in {el:.1f} s", file=sys.stderr, flush=True)
        out.append({"case": name, "kappa": kappa, "sem": guess == E.GUESS_SEM,
                    "total_iterations": st["iters_total"], "solves": st["n_solves"],
                    "seconds": el, "resid_max": st["resid_max"],
                    "paper_total_iterations": paper_its, "paper_hours": paper_h})
    base = out[0]["total_iterations"]
    for o in out:
        o["iterations_vs_case1"] = o["total_iterations"] / base
    print(json.dumps({"metric": "total GMRES iterations, Table 1 cases (prismatic rod)",
                      "n_elements": len(tri), "n_dof": N, "n_f": n_f, "gmres_tol": 1e-5,
                      "precond": "leaf block-diagonal", "operator": "H-matrix, ACA 1e-5",
                      "paper_context": "pFFT BEM, 12,800 triangles, one Xeon 3.0 GHz (Sec. 5.1)",
                      "cases": out}), flush=True)


def rod_long(args):
    """Sec. 5.1, the long-time run: the prismatic rod (3 x 1 x 1, nu = 0, fixed
    end, step traction at the free end) over a window of T = 0.035 s with
    N_w = 512 (257 frequency solves), kappa = 4 (eq. ewm-k), the least-squares
    extrapolation with K = 4, GMRES 1e-5, leaf block-diagonal preconditioner,
    ACA 1e-5.  In the units of rod-table1 (mu = rho = 1, T = 26.79 L / c for
    the paper's 0.0155 s) the window is T = 60.49 L / c.  Reports the time,
    the iterations and the end displacement against the 1-D bar's closed form
    (a triangle wave) and against that closed form passed through the same
    damped transform and window (which isolates the spatial error)."""
    import torch
    from paper_1212_3032_amd import ewbem as E
    from synth import box_mesh, ramp_history

    L = 3.0
    n = args.rod_div
    xyz, tri, face = box_mesh((L, 1, 1), (3 * n, n, n), origin=(0, -0.5, -0.5))
    bc = (face == 0).astype(np.int32)
    given = np.zeros((len(tri), 3))
    given[face == 1, 0] = -1.0
    c_bar = np.sqrt(2.0)
    period = 26.79 * L / c_bar * (0.035 / 0.0155)
    n_f = 512
    hist = ramp_history(n_f, period, 0.0)
    N = 3 * len(tri)
    sigma = 4.0 * np.log(10.0) / period
    c = E.Context(0)
    c.set_mesh(xyz, tri, exterior=False)
    c.set_material(1.0, 1.0, 0.0)
    c.set_time(period, n_f, sigma, E.WINDOW_HANN)
    c.set_load_mixed(bc, given, hist)
    c.set_operator(kind=E.OP_HMAT, leaf_size=64, eta_adm=1.0, aca_tol=1e-5)
    c.set_solver(tol=1e-5, guess=E.GUESS_SEM, sem_k=4, precond=E.PREC_LEAF, maxit=2000)
    u = torch.zeros(n_f * N, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = c.solve_transient(u, allow_noconv=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    c.close()
    # end displacement (mean over the loaded face, along -x: the traction pulls along -x)
    U = u.cpu().numpy().reshape(n_f, len(tri), 3)
    uL = -U[:, face == 1, 0].mean(axis=1)
    t = np.arange(n_f) * period / n_f
    mat = dict(rho=1.0, mu=1.0, nu=0.0)
    E_mod = 2.0
    tau = np.mod(t, 4 * L / c_bar)
    exact = c_bar * np.where(tau <= 2 * L / c_bar, tau, 4 * L / c_bar - tau) / E_mod
    # the closed form through the same transform: H(s) = c/(E s) tanh(s L / c) times the damped
    # DFT of the sampled step, conjugate-filled, Hann window, de-damped
    k = np.arange(n_f // 2 + 1)
    s_k = sigma + 2j * np.pi * k / period
    dt = period / n_f
    ph = np.array([np.sum(np.exp(-sigma * np.arange(n_f) * dt) * hist * np.exp(-2j * np.pi * kk * np.arange(n_f) / n_f))
                   for kk in k]) / n_f
    Hs = (c_bar / (E_mod * s_k)) * np.tanh(s_k * L / c_bar) * ph
    W = 0.5 * (1 + np.cos(2 * np.pi * k / n_f))
    full = np.zeros(n_f, complex)
    full[:n_f // 2 + 1] = W * Hs
    full[n_f // 2 + 1:] = np.conj((W * Hs)[1:n_f // 2][::-1])
    mft_exact = np.real(np.exp(sigma * t) * np.fft.ifft(full) * n_f)
    q = n_f // 4
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    print(json.dumps({
        "metric": "long-time run of Sec. 5.1 (prismatic rod, T = 0.035 s, N_w = 512)",
        "value": st["n_solves"] / el, "unit": "freq-solves/s", "n_gpus": 1, "seconds": el,
        "n_elements": len(tri), "n_dof": N, "n_f": n_f, "period_L_over_c": period * c_bar / L,
        "solves": st["n_solves"], "gmres_iters_total": st["iters_total"],
        "gmres_iters_per_solve": st["iters_total"] / st["n_solves"], "resid_max": st["resid_max"],
        "end_displacement_rel_l2_vs_closed_form": rel(uL, exact),
        "end_displacement_rel_l2_vs_transformed_closed_form": rel(uL, mft_exact),
        "by_quarter_vs_transformed_closed_form": [rel(uL[i * q:(i + 1) * q], mft_exact[i * q:(i + 1) * q])
                                                  for i in range(4)],
        "paper_context": "257 solves, dt = 6.84e-6 s; no timing given (Sec. 5.1)",
    }), flush=True)


def learned_workload(args):
    """The level-5 cavity under spherical-harmonic pressure loads (sums of 4
    real harmonics up to degree 6, N(0, 1) coefficients): the guess is
    trained on the first --train-cases loads (untimed), then --steps
    held-out loads are solved twice, timed: plain FP64 (complex128 factors,
    least-squares extrapolation) and learned + FP32 (complex64 factors,
    FP64 Arnoldi and residuals, the trained guess as an extra column)."""
    import torch
    from paper_1212_3032_amd import ewbem as E
    from synth import config_inputs

    d = config_inputs(4, sub=args.sub)
    dev = torch.device("cuda:0")
    N, n_f = 3 * len(d["tri"]), d["n_f"]
    loads = d["loads"]
    n_tr = min(args.train_cases, len(d["train"]))
    held = d["held_out"][:args.steps]
    op = dict(kind=E.OP_HMAT, leaf_size=64, eta_adm=1.0, aca_tol=1e-5)

    def make(store, guess):
        c = E.Context(0)
        c.set_mesh(d["xyz"], d["tri"], exterior=True)
        m = d["material"]
        c.set_material(m["rho"], m["mu"], m["nu"])
        c.set_time(d["period"], n_f, d["sigma"], d["window"])
        c.set_load_pressure(loads[0], d["history"])
        c.set_operator(far_store=store, **op)
        c.set_solver(tol=1e-6, guess=guess, sem_k=3, precond=E.PREC_LEAF)
        return c

    u = torch.zeros(n_f * N, dtype=torch.float64, device=dev)
    cl = make(E.STORE_C64, E.GUESS_LEARNED)
    t = time.perf_counter()
    tr = cl.guess_train(loads[[d["train"][i] for i in range(n_tr)]], pressures=True, n_modes=args.learned_modes)
    t_train = time.perf_counter() - t
    print(f"# trained on {n_tr} loads in {t_train:.1f} s: pod energy {tr['pod_energy']:.8f}, "
          f"loss {tr['train_loss_first']:.3e} -> {tr['train_loss_last']:.3e}", file=sys.stderr, flush=True)
    cp = make(E.STORE_C128, E.GUESS_SEM)
    cp.set_load_pressure(loads[held[0]], d["history"])
    cp.solve_transient(u)  # warmup: the learned context was warmed by its training solves
    res = {}
    plain_u = {}  # held-out transients of the plain FP64 pass, for the error of the other
    for name, c in (("plain_fp64", cp), ("learned_fp32", cl)):
        tot = dict(its=0, solves=0, resid=0.0, guess=0.0, learned=0, t=0.0, t_gmres=0.0, err=0.0)
        for i in held:
            c.set_load_pressure(loads[i], d["history"])
            torch.cuda.synchronize()
            t = time.perf_counter()
            st = c.solve_transient(u)
            torch.cuda.synchronize()
            tot["t"] += time.perf_counter() - t
            tot["its"] += st["iters_total"]
            tot["solves"] += st["n_solves"]
            tot["resid"] = max(tot["resid"], st["resid_max"])
            tot["guess"] += st["guess_resid_sum"]
            tot["learned"] += st["guess_learned"]
            tot["t_gmres"] += st["t_gmres_ms"]
            if name == "plain_fp64":
                plain_u[i] = u.clone()
            else:
                tot["err"] = max(tot["err"], (torch.linalg.norm(u - plain_u[i]) / torch.linalg.norm(plain_u[i])).item())
            print(f"# {name} load {i}: {st['iters_total']} its, guess residual sum "
                  f"{st['guess_resid_sum']:.3e}", file=sys.stderr, flush=True)
        res[name] = {"value": tot["solves"] / tot["t"], "gmres_iters_per_solve": tot["its"] / tot["solves"],
                     "resid_max": tot["resid"], "guess_resid_mean": tot["guess"] / tot["solves"],
                     "learned_guesses": tot["learned"], "gmres_ms_per_solve": tot["t_gmres"] / tot["solves"],
                     "ms_per_step": 1000.0 * tot["t"] / len(held)}
        if name != "plain_fp64":
            res[name]["transient_rel_l2_vs_fp64_max"] = tot["err"]
    cl.close()
    cp.close()
    lf, pf = res["learned_fp32"], res["plain_fp64"]
    print(json.dumps({
        "metric": METRIC, "value": lf["value"], "unit": "freq-solves/s", "n_gpus": 1,
        "steps": len(held), "warmup": 1, "ms_per_step": lf["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+c64-factors+bf16-net", "data": "synthetic",
        "config": {"workload": d["name"] + " (held-out loads)", "n_dof": N, "n_f": n_f,
                   "train_loads": n_tr, "held_out_loads": [int(i) for i in held], "gmres_tol": 1e-6,
                   "aca_tol": 1e-5, "n_modes": args.learned_modes, "network": "3 x 256 GELU, bf16 products"},
        "plain_fp64": pf, "learned_fp32": lf, "speedup_vs_plain": lf["value"] / pf["value"],
        "training": {"seconds": t_train, "solves": tr["n_solves"], "pod_energy": tr["pod_energy"],
                     "loss_first": tr["train_loss_first"], "loss_last": tr["train_loss_last"]},
    }), flush=True)


def loads_workload(args):
    """The level-5 cavity under --n-loads spherical-harmonic pressure loads
    (the held-out loads of the learned workload first), complex128 factors,
    GMRES 1e-6: one transient per load (every frequency assembled once per
    load) against all loads through one frequency loop (assembled once for
    all).  Both on one context after a warm-up transient."""
    import torch
    from paper_1212_3032_amd import ewbem as E
    from synth import config_inputs

    d = config_inputs(4, sub=args.sub)
    dev = torch.device("cuda:0")
    N, n_f = 3 * len(d["tri"]), d["n_f"]
    order = list(d["held_out"]) + list(d["train"])
    pick = order[:args.n_loads]
    loads = d["loads"][pick]
    c = E.Context(0)
    c.set_mesh(d["xyz"], d["tri"], exterior=True)
    m = d["material"]
    c.set_material(m["rho"], m["mu"], m["nu"])
    c.set_time(d["period"], n_f, d["sigma"], d["window"])
    c.set_load_pressure(loads[0], d["history"])
    c.set_operator(kind=E.OP_HMAT, leaf_size=64, eta_adm=1.0, aca_tol=1e-5,
                   far_store=E.STORE_C64 if args.store == "c64" else E.STORE_C128, mv_mfma=args.mv_mfma)
    c.set_solver(tol=1e-6, guess=E.GUESS_SEM, sem_k=3, precond=E.PREC_LEAF)
    u1 = torch.zeros(n_f * N, dtype=torch.float64, device=dev)
    c.solve_transient(u1)  # warm-up: tree, tuning, first (cold) ACA
    torch.cuda.synchronize()
    seq = dict(t=0.0, solves=0, its=0, asm=0.0, gmres=0.0, mv_ms=0.0, mv_b=0.0, mv_n=0)
    for l in range(len(loads)):
        c.set_load_pressure(loads[l], d["history"])
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = c.solve_transient(u1)
        torch.cuda.synchronize()
        seq["t"] += time.perf_counter() - t
        seq["solves"] += st["n_solves"]
        seq["its"] += st["iters_total"]
        seq["asm"] += st["t_assemble_ms"]
        seq["gmres"] += st["t_gmres_ms"]
        seq["mv_ms"] += st["t_matvec_ms"]
        seq["mv_b"] += st["matvec_bytes_total"]
        seq["mv_n"] += st["matvecs_timed"]
        print(f"# one at a time, load {pick[l]}: {st['iters_total']} its", file=sys.stderr, flush=True)
    u = torch.zeros(len(loads) * n_f * N, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t = time.perf_counter()
    st = c.solve_transient_loads(loads, u, pressures=True)
    torch.cuda.synchronize()
    t_multi = time.perf_counter() - t
    c.close()
    v = st["n_solves"] / t_multi
    pv = seq["solves"] / seq["t"]
    # the last load's transient, alone and within the batch
    same = (torch.linalg.norm(u[(len(loads) - 1) * n_f * N:] - u1) / torch.linalg.norm(u1)).item()
    print(f"# {len(loads)} loads together: {st['iters_total']} its, {t_multi:.2f} s; one at a time "
          f"{seq['its']} its, {seq['t']:.2f} s; last load's transients differ by {same:.1e}",
          file=sys.stderr, flush=True)
    print(json.dumps({
        "metric": METRIC, "value": v, "unit": "freq-solves/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1000.0 * t_multi, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.store == "c128" else "f64+c64-factors", "data": "synthetic",
        "config": {"workload": d["name"] + f" ({len(loads)} pressure loads, one frequency loop)",
                   "n_dof": N, "n_f": n_f, "n_loads": len(loads), "gmres_tol": 1e-6, "aca_tol": 1e-5,
                   "eight_rhs_matvec": "FP64 matrix cores" if args.mv_mfma else "FP64 vector units"},
        "together": {"seconds": t_multi, "solves": st["n_solves"], "gmres_iters": st["iters_total"],
                     "assemble_ms": st["t_assemble_ms"], "gmres_ms": st["t_gmres_ms"],
                     "matvec_launches": st["matvecs_timed"], "matvec_ms": st["t_matvec_ms"],
                     "matvec_GBps": st["matvec_bytes_total"] / st["t_matvec_ms"] / 1e6},
        "one_at_a_time": {"value": pv, "seconds": seq["t"], "solves": seq["solves"], "gmres_iters": seq["its"],
                          "assemble_ms": seq["asm"], "gmres_ms": seq["gmres"], "matvec_launches": seq["mv_n"],
                          "matvec_ms": seq["mv_ms"], "matvec_GBps": seq["mv_b"] / seq["mv_ms"] / 1e6},
        "speedup": v / pv, "last_load_rel_diff": same,
    }), flush=True)


def scene_waves_workload(args):
    """The twelve-cavity scene (level 3 unless --sub) under --n-loads plane
    S-waves: seeded random directions with random normal polarisations, the
    scene's Ricker wavelet; complex64 factors at ACA 1e-4, GMRES 1e-6.  One
    transient per wave against all waves through one frequency loop, both on
    one context after a warm-up transient."""
    import torch
    from paper_1212_3032_amd import ewbem as E
    from synth import config_inputs

    sub = 3 if args.sub is None else args.sub
    d = config_inputs(5, sub=sub)
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(2012)
    dirs = rng.standard_normal((args.n_loads, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    pols = rng.standard_normal((args.n_loads, 3))
    pols -= (pols * dirs).sum(axis=1, keepdims=True) * dirs
    pols /= np.linalg.norm(pols, axis=1, keepdims=True)
    c = E.Context(0)
    c.set_mesh(d["xyz"], d["tri"], exterior=True)
    m = d["material"]
    c.set_material(m["rho"], m["mu"], m["nu"])
    c.set_time(d["period"], d["n_f"], d["sigma"], d["window"])
    c.set_load_incident_s([1.0, 0.0, 0.0], [0.0, 0.0, 1.0], 0.5, 13.0)
    c.set_operator(kind=E.OP_HMAT, leaf_size=64, eta_adm=1.0, aca_tol=1e-4, far_store=E.STORE_C64)
    c.set_solver(tol=1e-6, guess=E.GUESS_SEM, sem_k=3, precond=E.PREC_LEAF)
    N, n_f = 3 * len(d["tri"]), d["n_f"]
    u1 = torch.zeros(n_f * N, dtype=torch.float64, device=dev)
    c.solve_transient(u1)  # warm-up
    seq = dict(t=0.0, solves=0, its=0)
    for l in range(args.n_loads):
        c.set_load_incident_s(dirs[l], pols[l], 0.5, 13.0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = c.solve_transient(u1)
        torch.cuda.synchronize()
        seq["t"] += time.perf_counter() - t
        seq["solves"] += st["n_solves"]
        seq["its"] += st["iters_total"]
        print(f"# one at a time, wave {l}: {st['iters_total']} its", file=sys.stderr, flush=True)
    u = torch.zeros(args.n_loads * n_f * N, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t = time.perf_counter()
    st = c.solve_transient_incident_loads(dirs, pols, u)
    torch.cuda.synchronize()
    t_multi = time.perf_counter() - t
    c.close()
    same = (torch.linalg.norm(u[(args.n_loads - 1) * n_f * N:] - u1) / torch.linalg.norm(u1)).item()
    v, pv = st["n_solves"] / t_multi, seq["solves"] / seq["t"]
    print(f"# {args.n_loads} waves together: {st['iters_total']} its, {t_multi:.2f} s; one at a time "
          f"{seq['its']} its, {seq['t']:.2f} s; last wave's transients differ by {same:.1e}",
          file=sys.stderr, flush=True)
    print(json.dumps({
        "metric": "freq-solves/s, twelve-cavity scene under several incident waves (complex64 factors, 1e-6 residual)",
        "value": v, "unit": "freq-solves/s", "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": 1000.0 * t_multi,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+c64-factors",
        "data": "synthetic",
        "config": {"workload": d["name"].replace("sub5", f"sub{sub}") + f" ({args.n_loads} incident waves)",
                   "n_dof": N, "n_f": n_f, "n_waves": args.n_loads, "aca_tol": 1e-4, "gmres_tol": 1e-6},
        "together": {"seconds": t_multi, "solves": st["n_solves"], "gmres_iters": st["iters_total"],
                     "assemble_ms": st["t_assemble_ms"], "gmres_ms": st["t_gmres_ms"]},
        "one_at_a_time": {"value": pv, "seconds": seq["t"], "solves": seq["solves"], "gmres_iters": seq["its"]},
        "speedup": v / pv, "last_wave_rel_diff": same,
    }), flush=True)


def batch12_workload(args):
    """Twelve independent cavities (spheres and ellipsoids with semi-axes in
    [0.5, 2], icosphere levels 3-5, seeded pressure amplitudes; N_f = 128,
    complex64 factors, FP64 Arnoldi and residuals, ACA 1e-5, GMRES 1e-6).
    Timed twice from fresh contexts (tree, first cold ACA and all included):
    one problem at a time, and through the concurrent batch entry in waves
    of --wave problems (one context and stream each; a wave's contexts are
    closed before the next, which bounds the memory held at once)."""
    import torch
    from paper_1212_3032_amd import ewbem as E
    from synth import config_inputs

    probs = config_inputs(3, sub=args.sub)["problems"]
    dev = torch.device("cuda:0")

    def make(d, st=None, store=E.STORE_C64):
        c = E.Context(0, stream=None if st is None else st.cuda_stream)
        E.setup_from_inputs(c, d, op=dict(kind=E.OP_HMAT, leaf_size=64, eta_adm=1.0, aca_tol=1e-5,
                                          far_store=store),
                            solver=dict(tol=1e-6, guess=E.GUESS_SEM, sem_k=3, precond=E.PREC_LEAF))
        return c

    def out(d):
        return torch.zeros(d["n_f"] * 3 * len(d["tri"]), dtype=torch.float64, device=dev)

    small = min(probs, key=lambda d: len(d["tri"]))
    c = make(small)
    c.solve_transient(out(small))  # warmup: library and runtime start-up
    c.close()
    torch.cuda.synchronize()
    t = time.perf_counter()
    seq_solves = seq_its = 0
    for d in probs:
        c = make(d)
        st = c.solve_transient(out(d))
        free, total = torch.cuda.mem_get_info()
        c.close()
        seq_solves += st["n_solves"]
        seq_its += st["iters_total"]
        print(f"# one at a time: {d['name']} {st['iters_total']} its, {(total - free) / 1e9:.0f} GB in use",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t
    # waves with the sizes dealt round-robin, largest first
    order = sorted(range(len(probs)), key=lambda i: -len(probs[i]["tri"]))
    n_waves = (len(probs) + args.wave - 1) // args.wave
    waves = [[order[j] for j in range(w, len(order), n_waves)] for w in range(n_waves)]
    t = time.perf_counter()
    bat_solves = bat_its = 0
    resid = 0.0
    u_bat = {}
    for w in waves:
        streams = [torch.cuda.Stream() for _ in w]
        ctxs = [make(probs[i], st) for i, st in zip(w, streams)]
        for i in w:
            u_bat[i] = out(probs[i])
        st = E.batch_solve_transient(ctxs, [u_bat[i] for i in w], per_launch=16 if not args.lockstep else len(w),
                                     lockstep=args.lockstep)
        torch.cuda.synchronize()
        free, total = torch.cuda.mem_get_info()
        for c in ctxs:
            c.close()
        bat_solves += st["n_solves"]
        bat_its += st["iters_total"]
        resid = max(resid, st["resid_max"])
        print(f"# wave {[probs[i]['name'] for i in w]}: {st['iters_total']} its; device memory in use "
              f"before closing {(total - free) / 1e9:.0f} GB", file=sys.stderr, flush=True)
    t_bat = time.perf_counter() - t
    err64 = None
    if args.fp64_reference:
        err64 = 0.0
        for i, d in enumerate(probs):
            c = make(d, store=E.STORE_C128)
            ref = out(d)
            c.solve_transient(ref)
            c.close()
            e = (torch.linalg.norm(u_bat[i] - ref) / torch.linalg.norm(ref)).item()
            err64 = max(err64, e)
            print(f"# {d['name']}: complex64 transient vs complex128 {e:.2e}", file=sys.stderr, flush=True)
    n_dofs = [3 * len(d["tri"]) for d in probs]
    print(json.dumps({
        "metric": "freq-solves/s, twelve uneven cavities (complex64 factors, 1e-6 residual)",
        "value": bat_solves / t_bat, "unit": "freq-solves/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1000.0 * t_bat, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+c64-factors", "data": "synthetic",
        "config": {"workload": "12-cavities-batched", "n_dof": n_dofs, "n_dof_total": int(sum(n_dofs)),
                   "n_f": probs[0]["n_f"], "aca_tol": 1e-5, "gmres_tol": 1e-6,
                   "waves": [[probs[i]["name"] for i in w] for w in waves],
                   "batch": "lock-step, one concatenated matvec per Arnoldi step" if args.lockstep
                            else "concurrent host threads, one stream per problem"},
        "one_at_a_time": {"value": seq_solves / t_seq, "ms": 1000.0 * t_seq,
                          "gmres_iters_per_solve": seq_its / seq_solves},
        "concurrent": {"value": bat_solves / t_bat, "ms": 1000.0 * t_bat,
                       "gmres_iters_per_solve": bat_its / bat_solves, "resid_max": resid,
                       "transient_rel_l2_vs_fp64_max": err64},
        "speedup_concurrent": (bat_solves / t_bat) / (seq_solves / t_seq),
    }), flush=True)


def scene_workload(args):
    """Twelve spherical cavities at seeded centres in a 20^3 box, one mesh,
    scattering a plane S-wave along +x polarised along z (Ricker, f_c = 0.5,
    peak crossing x = -10 at t = 1.5 / f_c); T = 32, N_f = 256 (129 solves),
    sigma = 8 / T, complex64 factors at ACA 1e-4, FP64 Arnoldi and residuals,
    GMRES 1e-6.  Level 3 by default (46,080 unknowns)."""
    import torch
    from paper_1212_3032_amd import ewbem as E
    from synth import config_inputs

    sub = 3 if args.sub is None else args.sub
    per_freq = args.per_frequency or sub >= 5
    d = config_inputs(5, sub=sub)
    dev = torch.device("cuda:0")
    t_setup = time.perf_counter()
    c = E.Context(0)
    c.set_mesh(d["xyz"], d["tri"], exterior=True)
    m = d["material"]
    c.set_material(m["rho"], m["mu"], m["nu"])
    c.set_time(d["period"], d["n_f"], d["sigma"], d["window"])
    c.set_load_incident_s([1.0, 0.0, 0.0], [0.0, 0.0, 1.0], 0.5, 13.0, total=args.total_field)
    c.set_operator(kind=E.OP_HMAT, leaf_size=64, eta_adm=1.0, aca_tol=1e-4, far_store=E.STORE_C64,
                   aca_batch_mb=args.aca_batch_mb)
    c.set_solver(tol=1e-6, guess=E.GUESS_SEM, sem_k=3, precond=E.PREC_LEAF)
    N = 3 * len(d["tri"])
    info0 = c.info()
    print(f"# scene level {sub}: {N} unknowns, {info0['n_near']} near / {info0['n_far']} far blocks, "
          f"near field {16 * info0['near_entries'] / 1e9:.1f} GB (set-up {time.perf_counter() - t_setup:.1f} s)",
          file=sys.stderr, flush=True)
    u = torch.zeros(d["n_f"] * N, dtype=torch.float64, device=dev)
    nk = d["n_f"] // 2 + 1

    def one_transient():
        if not per_freq:
            return c.solve_transient(u)
        spec = torch.zeros(nk * N, dtype=torch.complex128, device=dev)
        tot = None
        t0 = time.perf_counter()
        for k in range(nk):
            st = c.solve_frequency(k, spec[k * N:(k + 1) * N])
            tot = st if tot is None else {q: (max(tot[q], v) if q in ("resid_max", "iters_max", "rank_max")
                                              else v if q in ("matvec_bytes", "stored_bytes", "n_near", "n_far",
                                                              "rank_sum") else tot[q] + v) for q, v in st.items()}
            print(f"# k={k}: {st['iters_total']} its, resid {st['resid_max']:.1e}, rank max {st['rank_max']}, "
                  f"stored {st['stored_bytes'] / 1e9:.1f} GB, {time.perf_counter() - t0:.0f} s",
                  file=sys.stderr, flush=True)
        c.mft_inverse(spec, u)
        return tot

    for _ in range(args.warmup):
        one_transient()
    torch.cuda.synchronize()
    t = time.perf_counter()
    tot = None
    for _ in range(args.steps):
        st = one_transient()
        tot = st if tot is None else {k: (max(tot[k], v) if k in ("resid_max", "iters_max", "rank_max")
                                          else v if k in ("matvec_bytes", "stored_bytes", "n_near", "n_far",
                                                          "rank_sum") else tot[k] + v) for k, v in st.items()}
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    info = c.info()
    c.close()
    err64 = None
    if args.fp64_reference:
        c = E.Context(0)
        c.set_mesh(d["xyz"], d["tri"], exterior=True)
        c.set_material(m["rho"], m["mu"], m["nu"])
        c.set_time(d["period"], d["n_f"], d["sigma"], d["window"])
        c.set_load_incident_s([1.0, 0.0, 0.0], [0.0, 0.0, 1.0], 0.5, 13.0, total=args.total_field)
        c.set_operator(kind=E.OP_HMAT, leaf_size=64, eta_adm=1.0, aca_tol=1e-4, far_store=E.STORE_C128)
        c.set_solver(tol=1e-6, guess=E.GUESS_SEM, sem_k=3, precond=E.PREC_LEAF)
        ref = torch.zeros_like(u)
        for _ in range(args.warmup + args.steps):  # the same sequence of warm-started passes
            c.solve_transient(ref)
        c.close()
        err64 = (torch.linalg.norm(u - ref) / torch.linalg.norm(ref)).item()
        print(f"# complex64 transient vs complex128 {err64:.2e}", file=sys.stderr, flush=True)
    n = tot["n_solves"]
    mv_s = tot["t_matvec_ms"] / 1000.0
    print(json.dumps({
        "metric": "freq-solves/s, twelve-cavity scattering scene (complex64 factors, 1e-6 residual)",
        "value": n / el, "unit": "freq-solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1000.0 * el / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+c64-factors", "data": "synthetic",
        "config": {"workload": d["name"].replace("sub5", f"sub{sub}"), "n_dof": N, "n_f": d["n_f"],
                   "period": d["period"], "sigma": d["sigma"], "aca_tol": 1e-4, "gmres_tol": 1e-6,
                   "far_blocks": info["n_far"], "near_blocks": info["n_near"],
                   "formulation": "total field (b = u_inc)" if args.total_field else "scattered field (b = U t_sc)",
                   "aca_batch_mb": args.aca_batch_mb, "driven_per_frequency": per_freq},
        "gmres_iters_per_solve": tot["iters_total"] / n, "resid_max": tot["resid_max"],
        "transient_rel_l2_vs_fp64": err64,
        "matvec_GBps": tot["matvec_bytes_total"] / mv_s / 1e9 if mv_s > 0 else None,
        "stored_operator_GB": tot["stored_bytes"] / 1e9, "rank_max": tot["rank_max"],
        "phases_ms_per_step": {"assembly_ms": tot["t_assemble_ms"] / args.steps,
                               "aca_kernels_ms": tot["t_aca_ms"] / args.steps,
                               "gmres_ms": tot["t_gmres_ms"] / args.steps,
                               "guess_ms": tot["t_guess_ms"] / args.steps},
    }), flush=True)


def cpu_baseline(args):
    """The oracle (dense assembly + LU) on the host cores, on a bounded sample
    of the same workload: ``cpu_rows`` element rows of T and U at level 5
    and a full LU at level 3, scaled to one frequency solve at 61,440
    unknowns (assembly linear in rows, LU cubic in N)."""
    from threadpoolctl import threadpool_info
    from oracle import bem, kernels as K, mft
    from synth import config_inputs

    d = config_inputs(2, sub=args.sub)
    mat = K.material(**d["material"])
    g = bem.geometry(d["xyz"], d["tri"])
    s = mft.freq_grid(d["period"], d["n_f"], d["sigma"])[d["n_f"] // 4]
    rows = min(args.cpu_rows, g["ne"])
    t = time.perf_counter()
    bem.assemble_rows(g, s, mat, np.arange(rows))
    t_rows = time.perf_counter() - t
    t_asm = t_rows * g["ne"] / rows
    d3 = config_inputs(2, sub=3)
    g3 = bem.geometry(d3["xyz"], d3["tri"])
    A3, U3 = bem.assemble_dense(g3, s, mat)
    b3 = U3 @ bem.traction_from_pressure(g3, d3["pressure"])
    t = time.perf_counter()
    np.linalg.solve(A3, b3)
    t_lu3 = time.perf_counter() - t
    N = 3 * g["ne"]
    t_lu = t_lu3 * (N / (3 * g3["ne"])) ** 3
    threads = 1
    blas = []
    for info in threadpool_info():
        if info.get("user_api") == "blas":
            threads = max(threads, info.get("num_threads", 1))
            blas.append(f"{info.get('internal_api')} {info.get('version')} ({info.get('architecture')})")
    return {
        "value": 1.0 / (t_asm + t_lu), "unit": "freq-solves/s", "cores": threads,
        "kind": "oracle",
        "sample": (f"dense oracle: {rows} element rows of T and U at N={N} in {t_rows:.1f} s "
                   f"(scaled to all rows: {t_asm:.0f} s) + LAPACK LU at N={3 * g3['ne']} in "
                   f"{t_lu3:.2f} s (scaled by N^3: {t_lu:.0f} s); extrapolated, one frequency"),
        "host_cpus": len(os.sched_getaffinity(0)),
        "blas": "; ".join(blas) or "unknown",
    }


def time_transients(ctx, u, n, ref=None):
    """n transients on ctx (its current load), each bracketed by device
    synchronisations; totals, and the largest relative L2 difference of the
    transient from ref[i] when given."""
    import torch
    tot = dict(t=0.0, solves=0, its=0, resid=0.0, guess=0.0, learned=0, gmres=0.0, err=0.0, u=[])
    for i in range(n):
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = ctx.solve_transient(u)
        torch.cuda.synchronize()
        tot["t"] += time.perf_counter() - t
        tot["solves"] += st["n_solves"]
        tot["its"] += st["iters_total"]
        tot["resid"] = max(tot["resid"], st["resid_max"])
        tot["guess"] += st["guess_resid_sum"]
        tot["learned"] += st["guess_learned"]
        tot["gmres"] += st["t_gmres_ms"]
        if ref is not None:
            tot["err"] = max(tot["err"], (torch.linalg.norm(u - ref[i]) / torch.linalg.norm(ref[i])).item())
        tot["u"].append(u.clone())
    return tot


def leg_summary(tot, n):
    return {"value": tot["solves"] / tot["t"], "unit": "freq-solves/s", "transients": n,
            "ms_per_transient": 1000.0 * tot["t"] / max(1, n),
            "gmres_iters_per_solve": tot["its"] / max(1, tot["solves"]),
            "guess_resid_mean": tot["guess"] / max(1, tot["solves"]), "resid_max": tot["resid"],
            "gmres_ms_per_solve": tot["gmres"] / max(1, tot["solves"])}


def cavity_variants(args, held_loads):
    """Runs on the main context after its timed steps: the quadratic
    extrapolation variant, then the plain FP64 leg of the learned
    comparison on held-out spherical-harmonic loads."""
    from paper_1212_3032_amd import ewbem as E

    def after(ctx, d, u):
        out = {}
        if args.variant_steps > 0:
            ctx.set_solver(tol=1e-6, guess=E.GUESS_QUAD, sem_k=3, precond=E.PREC_LEAF)
            tot = time_transients(ctx, u, args.variant_steps)
            out["quad"] = leg_summary(tot, args.variant_steps)
            print(f"# quadratic extrapolation: {tot['its']} its over {tot['solves']} solves",
                  file=sys.stderr, flush=True)
        if held_loads is not None:
            loads, hist = held_loads
            ctx.set_solver(tol=1e-6, guess=E.GUESS_SEM, sem_k=3, precond=E.PREC_LEAF)
            tot = dict(t=0.0, solves=0, its=0, resid=0.0, guess=0.0, learned=0, gmres=0.0, err=0.0, u=[])
            for p in loads:
                ctx.set_load_pressure(p, hist)
                t1 = time_transients(ctx, u, 1)
                for k in ("t", "solves", "its", "guess", "learned", "gmres"):
                    tot[k] += t1[k]
                tot["resid"] = max(tot["resid"], t1["resid"])
                tot["u"] += t1["u"]
            out["plain_held"] = tot
            print(f"# plain FP64 on held-out loads: {tot['its']} its over {tot['solves']} solves",
                  file=sys.stderr, flush=True)
        return out
    return after


def learned_leg(args, d4, held, plain):
    """The learned + FP32 leg: complex64 far factors (FP64 Arnoldi and
    residuals) and the trained guess, on the held-out loads the plain leg
    solved; training (untimed) on the first --learned-train loads."""
    from paper_1212_3032_amd import ewbem as E
    import torch

    N, n_f = 3 * len(d4["tri"]), d4["n_f"]
    c = E.Context(0)
    c.set_mesh(d4["xyz"], d4["tri"], exterior=True)
    m = d4["material"]
    c.set_material(m["rho"], m["mu"], m["nu"])
    c.set_time(d4["period"], n_f, d4["sigma"], d4["window"])
    c.set_load_pressure(d4["loads"][held[0]], d4["history"])
    c.set_operator(kind=E.OP_HMAT, leaf_size=64, eta_adm=1.0, aca_tol=1e-5, far_store=E.STORE_C64)
    c.set_solver(tol=1e-6, guess=E.GUESS_LEARNED, sem_k=3, precond=E.PREC_LEAF)
    tr_ids = d4["train"][:args.learned_train]
    t = time.perf_counter()
    tr = c.guess_train(d4["loads"][tr_ids], pressures=True, n_modes=args.learned_modes)
    t_train = time.perf_counter() - t
    print(f"# learned guess trained on {len(tr_ids)} loads in {t_train:.1f} s", file=sys.stderr, flush=True)
    u = torch.zeros(n_f * N, dtype=torch.float64, device="cuda:0")
    tot = dict(t=0.0, solves=0, its=0, resid=0.0, guess=0.0, learned=0, gmres=0.0, err=0.0, u=[])
    for j, i in enumerate(held):
        c.set_load_pressure(d4["loads"][i], d4["history"])
        t1 = time_transients(c, u, 1, ref=[plain["u"][j]])
        for k in ("t", "solves", "its", "guess", "learned", "gmres"):
            tot[k] += t1[k]
        tot["resid"] = max(tot["resid"], t1["resid"])
        tot["err"] = max(tot["err"], t1["err"])
    c.close()
    pl = leg_summary(plain, len(held))
    le = leg_summary(tot, len(held))
    le["learned_guesses"] = tot["learned"]
    le["transient_rel_l2_vs_fp64_max"] = tot["err"]
    print(f"# learned + FP32 on held-out loads: {tot['its']} its over {tot['solves']} solves, "
          f"transient vs FP64 {tot['err']:.2e}", file=sys.stderr, flush=True)
    return {
        "workload": d4["name"].replace("sub5", f"sub{args.sub}") if args.sub else d4["name"],
        "held_out_loads": [int(i) for i in held], "train_loads": [int(i) for i in tr_ids],
        "plain_fp64": dict(pl, guess="LS extrapolation K=3", far_store="c128"),
        "learned_fp32": dict(le, guess="learned column + LS extrapolation K=3", far_store="c64",
                             n_modes=args.learned_modes, network="3 x 256 GELU, bf16 products"),
        "speedup_vs_plain": le["value"] / pl["value"],
        "training": {"seconds": t_train, "solves": tr["n_solves"], "pod_energy": tr["pod_energy"],
                     "loss_first": tr["train_loss_first"], "loss_last": tr["train_loss_last"]},
    }


def main():
    args = parse()
    if args.traffic_summary:
        fetch_dir, write_dir, run_log = args.traffic_summary
        traffic_summary(fetch_dir, write_dir, run_log=run_log)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: --gpus must be 1 (the split of the frequencies "
                                   "over several GPUs is a design, not built)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "rod-table1":
        rod_table1(args)
        return
    if args.workload == "rod-long":
        rod_long(args)
        return
    if args.workload == "learned":
        learned_workload(args)
        return
    if args.workload == "batch12":
        batch12_workload(args)
        return
    if args.workload == "scene":
        scene_workload(args)
        return
    if args.workload == "loads":
        loads_workload(args)
        return
    if args.workload == "scene-waves":
        scene_waves_workload(args)
        return
    if args.copy_probe:
        copy_probe()
    d4 = held = None
    if args.learned_train > 0 and args.learned_held > 0:
        from synth import config_inputs
        d4 = config_inputs(4, sub=args.sub)
        held = d4["held_out"][:args.learned_held]
    d, N, elapsed, st, var = run_gpu(
        args, args.store,
        after=cavity_variants(args, None if d4 is None else ([d4["loads"][i] for i in held], d4["history"])))
    u_ref = st.pop("u_last")
    solves = st["n_solves"]
    value = solves / elapsed
    ms_step = 1000.0 * elapsed / args.steps
    mv_time_s = st["t_matvec_ms"] / 1000.0
    mv_gbs = st["matvec_bytes_total"] / mv_time_s / 1e9 if mv_time_s > 0 else 0.0
    per_launch_ms = st["t_matvec_ms"] / max(1, st["matvecs_timed"])
    bytes_per_launch = st["matvec_bytes_total"] / max(1, st["matvecs_timed"])
    phases = {
        "assembly_ms": st["t_assemble_ms"] / args.steps,
        "near_self_kernels_ms": st["t_near_ms"] / args.steps,
        "aca_kernels_ms": st["t_aca_ms"] / args.steps,
        "rhs_kernels_ms": st["t_rhs_ms"] / args.steps,
        "guess_ms": st["t_guess_ms"] / args.steps,
        "gmres_ms": st["t_gmres_ms"] / args.steps,
        "matvec_kernels_ms": st["t_matvec_ms"] / args.steps,
        "post_ms": st["t_post_ms"] / args.steps,
    }
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "freq-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.store == "c128" else "f64+c64-factors",
        "data": "synthetic",
        "config": {
            "workload": d["name"], "n_dof": N, "n_elements": len(d["tri"]), "n_f": d["n_f"],
            "freq_solves_per_step": solves // args.steps, "sigma": d["sigma"], "period": d["period"],
            "leaf": 64, "eta_adm": 1.0, "aca_tol": 1e-5, "gmres_tol": 1e-6,
            "guess": "least-squares extrapolation over the 3 previous solutions (Sec. 4.2)",
            "precond": "leaf block-diagonal", "far_store": args.store, "arith": "complex128",
            "aca_block_starts_per_frequency": {"warm": st["aca_warm_blocks"] / max(1, solves),
                                               "cold": st["aca_cold_blocks"] / max(1, solves)},
        },
        "roofline": {
            "kernel": "H-matrix matvec (k_far_vt + k_hmv + k_hmv_reduce)",
            "bound": "hbm", "achieved": mv_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": mv_gbs / HBM_PEAK_GBS, "traffic": traffic_from_profiles(bytes_per_launch),
            "algorithmic_bytes_per_launch": bytes_per_launch, "avg_launch_ms": per_launch_ms,
            "launches": st["matvecs_timed"],
        },
        "phases_ms_per_step": phases,
        "rates_freq_solves_per_s": {
            "end_to_end": value,
            "assembly_only": solves / (st["t_assemble_ms"] / 1000.0),
            "solve_only": solves / ((st["t_guess_ms"] + st["t_gmres_ms"]) / 1000.0)},
        "matvec_shapes": st["matvec_shapes"],
        "gmres_iters_per_solve": st["iters_total"] / max(1, solves),
        "resid_max": st["resid_max"],
        "stored_operator_GB": st["stored_bytes"] / 1e9,
        "device_memory_GB": st["device_memory_GB"],
        "library_memory_GB": st["library_memory_GB"],
        "far_blocks": st["n_far"], "near_blocks": st["n_near"], "rank_max": st["rank_max"],
    }
    if not args.no_read_probe:
        rp = read_probe()
        out["roofline"]["stream_read_probe_GBps"] = rp
        out["roofline"]["frac_of_stream_read_probe"] = mv_gbs / rp
    if args.c64_variant and args.store == "c128":
        _, _, el2, st2, _ = run_gpu(args, "c64")
        u2 = st2.pop("u_last")
        out["c64_factors"] = {
            "value": st2["n_solves"] / el2,
            "matvec_GBps": st2["matvec_bytes_total"] / (st2["t_matvec_ms"] / 1000.0) / 1e9,
            "gmres_iters_per_solve": st2["iters_total"] / max(1, st2["n_solves"]),
            "resid_max": st2["resid_max"],
            "transient_rel_l2_vs_fp64": float(np.linalg.norm(u2 - u_ref) / np.linalg.norm(u_ref)),
        }
    if not args.no_pipeline_variant and args.variant_steps > 0:
        _, _, el3, st3, _ = run_gpu(args, args.store, pipeline=1)
        u3 = st3.pop("u_last")
        out["pipelined"] = {
            "value": st3["n_solves"] / el3,
            "ms_per_step": 1000.0 * el3 / args.steps,
            "note": "the next frequency's ACA on a second stream while GMRES solves the current one "
                    "(ewbem_solver_opts.pipeline); same arithmetic, a second far-factor slot",
            "transient_rel_l2_vs_sequential": float(np.linalg.norm(u3 - u_ref) / np.linalg.norm(u_ref)),
            "matvec_GBps": st3["matvec_bytes_total"] / (st3["t_matvec_ms"] / 1000.0) / 1e9,
            "gmres_iters_per_solve": st3["iters_total"] / max(1, st3["n_solves"]),
        }
    if "quad" in var:
        out["quad_variant"] = dict(var["quad"], guess="quadratic extrapolation 3 a1 - 3 a2 + a3 (no operator "
                                                      "products; inside the span of the least-squares one)")
    if "plain_held" in var:
        out["learned_fp32"] = learned_leg(args, d4, held, var["plain_held"])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
