"""No kernel reads device memory that no kernel wrote.

With EWBEM_POISON_ALLOC set in its environment (read once per process) the
library fills every new floating-point buffer with all-ones bytes, a NaN
pattern.  A child process runs a few whole paths that way -- dense
transients with the least-squares and the quadratic extrapolation, an
H-matrix transient with warm-started ACA, two loads through one frequency
loop, and the same context's own transient after them -- and its results
must hold no NaN and equal those of this process, which runs the same paths
on ordinary allocations (autotuning off, so both take the same task shapes).

A fresh process usually receives zeroed memory, so such a read can go
unnoticed until an allocation recycles memory that held NaN; the
extrapolation once formed its guess over every history slot, unwritten ones
included (with zero coefficients, which a NaN turns into NaN)."""

import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NF, PERIOD = 16, 8.0


def run_paths(out_path):
    """Every path once; the transients and spectra into an .npz."""
    import torch

    sys.path.insert(0, ROOT)
    from paper_1212_3032_amd import ewbem as E
    from synth import icosphere, ramp_history, sh_pressure

    dev = torch.device("cuda:0")
    res = {}

    def ctx(xyz, tri, p, op, guess):
        c = E.Context(0)
        c.set_mesh(xyz, tri, exterior=True)
        c.set_material(1.0, 1.0, 0.25)
        c.set_time(PERIOD, NF, 6.0 / PERIOD, 1)
        c.set_load_pressure(p, ramp_history(NF, PERIOD, 0.05))
        c.set_operator(**op)
        c.set_solver(tol=1e-8, guess=guess)
        return c

    rng = np.random.default_rng(77)
    for sub, op in ((2, dict(kind=E.OP_DENSE, autotune=0)),
                    (3, dict(kind=E.OP_HMAT, leaf_size=64, eta_adm=1.0, aca_tol=1e-6, autotune=0))):
        xyz, tri = icosphere(sub)
        N = 3 * len(tri)
        p = sh_pressure(xyz, tri, rng)[0]
        guesses = ((E.GUESS_SEM, "sem"), (E.GUESS_QUAD, "quad")) if sub == 2 else ((E.GUESS_SEM, "sem"),)
        for guess, name in guesses:
            c = ctx(xyz, tri, p, op, guess)
            u = torch.zeros(NF * N, dtype=torch.float64, device=dev)
            c.solve_transient(u)
            res[f"sub{sub}_{name}"] = u.cpu().numpy()
            c.close()
        if sub == 3:
            loads = np.array([sh_pressure(xyz, tri, rng)[0] for _ in range(2)])
            c = ctx(xyz, tri, p, op, E.GUESS_SEM)
            u = torch.zeros(2 * NF * N, dtype=torch.float64, device=dev)
            c.solve_transient_loads(loads, u, pressures=True)
            res["sub3_loads"] = u.cpu().numpy()
            u = torch.zeros(NF * N, dtype=torch.float64, device=dev)
            c.solve_transient(u)
            res["sub3_own_after_loads"] = u.cpu().numpy()
            c.close()
    np.savez(out_path, **res)


def test_no_read_of_unwritten_memory(tmp_path):
    ref_path = str(tmp_path / "plain.npz")
    poi_path = str(tmp_path / "poisoned.npz")
    run_paths(ref_path)
    env = dict(os.environ, EWBEM_POISON_ALLOC="1")
    code = f"import sys; sys.path.insert(0, {ROOT!r}); sys.path.insert(0, {os.path.dirname(__file__)!r}); " \
           f"import test_gpu_poison as t; t.run_paths({poi_path!r})"
    print("child: the same paths with poisoned allocations", flush=True)
    r = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    a, b = np.load(ref_path), np.load(poi_path)
    assert sorted(a.files) == sorted(b.files)
    for k in a.files:
        nan = int(np.isnan(b[k]).sum())
        d = float(np.linalg.norm(b[k] - a[k]) / np.linalg.norm(a[k])) if not nan else float("nan")
        print(f"  {k}: NaN entries {nan}, relative difference {d:.1e}", flush=True)
        assert nan == 0, k
        assert d <= 1e-12, k
