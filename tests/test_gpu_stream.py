"""The streamed far-field approximation (op.aca_batch_mb > 0): far blocks
approximated in batches through one complex128 work area, each batch
converted to complex64 as it finishes.  Each block's approximation does
not depend on which blocks share its launch, so the factors, and with them
every product and solution, must equal those of the unstreamed complex64
run bit for bit -- across warm-started frequencies and on a transient --
while the work area stays a fraction of the whole far field.  The
unstreamed complex64 path is itself checked against the oracle in
test_gpu_parity.py."""

import sys

import numpy as np
import pytest

from synth import config_inputs, icosphere, ramp_history, uniform_pressure

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _ctx(E, xyz, tri, batch_mb, n_f=32, tol=1e-6):
    c = E.Context(0)
    c.set_mesh(xyz, tri, exterior=True)
    c.set_material(1.0, 1.0, 0.25)
    c.set_time(8.0, n_f, 6.0 / 8.0, 1)
    c.set_load_pressure(uniform_pressure(len(tri), 1.0), ramp_history(n_f, 8.0, 0.05))
    c.set_operator(kind=E.OP_HMAT, leaf_size=64, eta_adm=1.0, aca_tol=tol, far_store=E.STORE_C64,
                   aca_batch_mb=batch_mb, autotune=0)
    c.set_solver(tol=1e-8, guess=E.GUESS_SEM)
    return c


def test_streamed_factors_equal_unstreamed():
    import torch
    from paper_1212_3032_amd import ewbem as E
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    xyz, tri = icosphere(3)
    N = 3 * len(tri)
    rng = np.random.default_rng(5)
    x = torch.tensor(rng.standard_normal(N) + 1j * rng.standard_normal(N), device=dev)
    a, b = _ctx(E, xyz, tri, 0), _ctx(E, xyz, tri, 4)
    for k in range(0, 17):
        sa, sb = a.assemble(k), b.assemble(k)
        assert sa["rank_sum"] == sb["rank_sum"]
        if k in (0, 1, 8, 16):
            ya = torch.zeros(N, dtype=torch.complex128, device=dev)
            yb = torch.zeros_like(ya)
            a.apply(x, ya)
            b.apply(x, yb)
            _say(f"k={k}: rank sum {sa['rank_sum']}, warm blocks {sb['aca_warm_blocks']}, "
                 f"max |diff| {float((ya - yb).abs().max()):.1e}")
            assert torch.equal(ya, yb)
    ua = torch.zeros(32 * N, dtype=torch.float64, device=dev)
    ub = torch.zeros_like(ua)
    a.solve_transient(ua)
    b.solve_transient(ub)
    assert torch.equal(ua, ub)
    a.close()
    b.close()


def test_streamed_scene_transient_equals_unstreamed():
    """The twelve-cavity scene at level 2 (11,520 unknowns) under the plane
    S-wave, total-field formulation: the transient of the streamed run with
    batches of 16 MiB equals the unstreamed one."""
    import torch
    from paper_1212_3032_amd import ewbem as E
    dev = torch.device("cuda:0")
    d = config_inputs(5, sub=2)
    N = 3 * len(d["tri"])
    us = []
    for mb in (0, 16):
        c = E.Context(0)
        c.set_mesh(d["xyz"], d["tri"], exterior=True)
        c.set_material(1.0, 1.0, 0.25)
        c.set_time(d["period"], 64, d["sigma"], 1)
        c.set_load_incident_s([1.0, 0.0, 0.0], [0.0, 0.0, 1.0], 0.5, 13.0, total=True)
        c.set_operator(kind=E.OP_HMAT, leaf_size=64, eta_adm=1.0, aca_tol=1e-4, far_store=E.STORE_C64,
                       aca_batch_mb=mb, autotune=0)
        c.set_solver(tol=1e-6, guess=E.GUESS_SEM)
        u = torch.zeros(64 * N, dtype=torch.float64, device=dev)
        st = c.solve_transient(u)
        _say(f"scene level 2, batch {mb} MiB: {st['iters_total']} its, warm blocks {st['aca_warm_blocks']}")
        us.append(u)
        c.close()
    assert torch.equal(us[0], us[1])
