"""Several problems solved concurrently (one context and one stream each)
give the same transients as the same problems solved one at a time: the
kernels are deterministic and the contexts share nothing.  The problems
are two of the 12-problem workload's kinds: a sphere and an ellipsoid of
the seeded radii and semi-axes.  The lock-step batch (one concatenated
matvec per Arnoldi step, replayed from a HIP graph) does the same
arithmetic per problem: its transients equal the lone solves' to rounding
(the concatenated phase-1 launch may take more factor columns per
wavefront than a problem's own, which changes the summation order only),
and match the oracle."""

import sys

import numpy as np
import pytest

from synth import ellipsoid, icosphere, ramp_history, uniform_pressure

pytestmark = pytest.mark.gpu


def _ctx(E, torch, xyz, tri, stream):
    c = E.Context(0, stream=stream.cuda_stream)
    c.set_mesh(xyz, tri, exterior=True)
    c.set_material(1.0, 1.0, 0.25)
    c.set_time(8.0, 32, 0.75, 1)
    c.set_load_pressure(uniform_pressure(len(tri)), ramp_history(32, 8.0, 0.05))
    c.set_operator(kind=E.OP_HMAT, leaf_size=64, eta_adm=1.0, aca_tol=1e-6)
    c.set_solver(tol=1e-8, guess=E.GUESS_SEM)
    return c


def test_batch_equals_one_at_a_time():
    import torch
    from paper_1212_3032_amd import ewbem as E
    probs = [icosphere(3), ellipsoid(3, (1.5, 0.8, 1.1))]
    streams = [torch.cuda.Stream() for _ in probs]
    single = []
    for (xyz, tri), s in zip(probs, streams):
        c = _ctx(E, torch, xyz, tri, s)
        u = torch.zeros(32 * 3 * len(tri), dtype=torch.float64, device="cuda:0")
        c.solve_transient(u)
        torch.cuda.synchronize()
        single.append(u.cpu().numpy())
        c.close()
    ctxs = [_ctx(E, torch, xyz, tri, s) for (xyz, tri), s in zip(probs, streams)]
    outs = [torch.zeros(32 * 3 * len(tri), dtype=torch.float64, device="cuda:0") for _, tri in probs]
    st = E.batch_solve_transient(ctxs, outs, per_launch=2)
    torch.cuda.synchronize()
    print(f"batch: {st['n_solves']} solves, {st['iters_total']} iterations", flush=True)
    sys.stdout.flush()
    assert st["n_solves"] == 2 * 17
    for u, ref in zip(outs, single):
        got = u.cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    for c in ctxs:
        c.close()
    with pytest.raises(E.EwbemError):
        c2 = _ctx(E, torch, *probs[0], streams[0])
        E.batch_solve_transient([c2, c2], [outs[0], outs[0]])


def test_batch_matches_oracle():
    """Each problem of a concurrent batch against the oracle's dense LU
    transient: a level-1 sphere and a level-1 ellipsoid (240 unknowns each)
    with small leaves so that the H-matrix has far blocks (ACA 1e-9), GMRES
    tol 1e-10; relative L2 1e-6 per problem (the FP64 bar; the ACA bound,
    30 x 1e-9, lies below it)."""
    import torch
    from oracle import solve as osolve
    from paper_1212_3032_amd import ewbem as E
    probs = [icosphere(1), ellipsoid(1, (1.4, 0.7, 1.0))]
    streams = [torch.cuda.Stream() for _ in probs]
    hist = ramp_history(32, 8.0, 0.05)
    ctxs, outs, refs = [], [], []
    for (xyz, tri), s in zip(probs, streams):
        c = E.Context(0, stream=s.cuda_stream)
        c.set_mesh(xyz, tri, exterior=True)
        c.set_material(1.0, 1.0, 0.25)
        c.set_time(8.0, 32, 0.75, 1)
        c.set_load_pressure(uniform_pressure(len(tri)), hist)
        c.set_operator(kind=E.OP_HMAT, leaf_size=4, eta_adm=1.0, aca_tol=1e-9)
        c.set_solver(tol=1e-10, guess=E.GUESS_SEM)
        assert c.info()["n_far"] > 0
        ctxs.append(c)
        outs.append(torch.zeros(32 * 3 * len(tri), dtype=torch.float64, device="cuda:0"))
        print(f"batch vs oracle: oracle transient of {len(tri)} elements", flush=True)
        refs.append(osolve.transient(xyz, tri, dict(rho=1.0, mu=1.0, nu=0.25), 8.0, 32, 0.75, 1,
                                     uniform_pressure(len(tri)), hist)["u"].reshape(-1))
    st = E.batch_solve_transient(ctxs, outs, per_launch=2)
    torch.cuda.synchronize()
    assert st["n_solves"] == 2 * 17
    for i, (u, ref) in enumerate(zip(outs, refs)):
        e = np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(ref)
        print(f"  problem {i}: transient error vs oracle {e:.3e}", flush=True)
        assert e < 1e-6
    for c in ctxs:
        c.close()


def test_lockstep_batch_equals_one_at_a_time():
    """Three problems of different sizes (two level-3 shapes and a level-2
    sphere, N_f 32, 32 and 16 -- the last leaves the lock-step early), one
    group: each transient within 1e-12 of its lone solve and the same
    iteration counts; a second call (new graphs, replayed again, each ACA
    warm-started from the first call's last frequency) matches a second lone
    transient the same way."""
    import torch
    from paper_1212_3032_amd import ewbem as E
    probs = [icosphere(3), ellipsoid(3, (1.5, 0.8, 1.1)), icosphere(2, radius=0.7)]
    nfs = [32, 32, 16]

    def make(xyz, tri, n_f):
        c = E.Context(0)
        c.set_mesh(xyz, tri, exterior=True)
        c.set_material(1.0, 1.0, 0.25)
        c.set_time(8.0, n_f, 0.75, 1)
        c.set_load_pressure(uniform_pressure(len(tri)), ramp_history(n_f, 8.0, 0.05))
        c.set_operator(kind=E.OP_HMAT, leaf_size=64, eta_adm=1.0, aca_tol=1e-6, far_store=E.STORE_C64,
                       autotune=0)  # the same matvec shapes for all
        c.set_solver(tol=1e-8, guess=E.GUESS_SEM)
        return c

    single, single2, its = [], [], []
    for (xyz, tri), n_f in zip(probs, nfs):
        c = make(xyz, tri, n_f)
        u = torch.zeros(n_f * 3 * len(tri), dtype=torch.float64, device="cuda:0")
        st = c.solve_transient(u)
        single.append(u.cpu().numpy())
        its.append(st["iters_total"])
        c.solve_transient(u)  # a second transient starts its ACA from the first one's last pivots
        single2.append(u.cpu().numpy())
        c.close()
    ctxs = [make(xyz, tri, n_f) for (xyz, tri), n_f in zip(probs, nfs)]
    outs = [torch.zeros(n_f * 3 * len(tri), dtype=torch.float64, device="cuda:0") for (_, tri), n_f in zip(probs, nfs)]
    print("lock-step batch of three problems", flush=True)
    st = E.batch_solve_transient(ctxs, outs, per_launch=3, lockstep=True)
    torch.cuda.synchronize()
    print(f"lock-step: {st['n_solves']} solves, {st['iters_total']} iterations (lone: {sum(its)})", flush=True)
    assert st["n_solves"] == 17 + 17 + 9
    assert st["iters_total"] == sum(its)
    first = [u.cpu().numpy() for u in outs]
    for got, ref in zip(first, single):
        e = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"  transient vs lone solve {e:.1e}", flush=True)
        assert e <= 1e-12
    E.batch_solve_transient(ctxs, outs, per_launch=3, lockstep=True)
    for u, ref in zip(outs, single2):
        got = u.cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    for c in ctxs:
        c.close()


def test_lockstep_batch_matches_oracle():
    """The lock-step batch against the oracle's dense LU transients (the
    problems of test_batch_matches_oracle, ACA 1e-9, GMRES 1e-10): 1e-6."""
    import torch
    from oracle import solve as osolve
    from paper_1212_3032_amd import ewbem as E
    probs = [icosphere(1), ellipsoid(1, (1.4, 0.7, 1.0))]
    hist = ramp_history(32, 8.0, 0.05)
    ctxs, outs, refs = [], [], []
    for xyz, tri in probs:
        c = E.Context(0)
        c.set_mesh(xyz, tri, exterior=True)
        c.set_material(1.0, 1.0, 0.25)
        c.set_time(8.0, 32, 0.75, 1)
        c.set_load_pressure(uniform_pressure(len(tri)), hist)
        c.set_operator(kind=E.OP_HMAT, leaf_size=4, eta_adm=1.0, aca_tol=1e-9)
        c.set_solver(tol=1e-10, guess=E.GUESS_SEM)
        ctxs.append(c)
        outs.append(torch.zeros(32 * 3 * len(tri), dtype=torch.float64, device="cuda:0"))
        refs.append(osolve.transient(xyz, tri, dict(rho=1.0, mu=1.0, nu=0.25), 8.0, 32, 0.75, 1,
                                     uniform_pressure(len(tri)), hist)["u"].reshape(-1))
    st = E.batch_solve_transient(ctxs, outs, per_launch=2, lockstep=True)
    assert st["n_solves"] == 2 * 17
    for i, (u, ref) in enumerate(zip(outs, refs)):
        e = np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(ref)
        print(f"  lock-step problem {i}: transient error vs oracle {e:.3e}", flush=True)
        assert e < 1e-6
    for c in ctxs:
        c.close()
