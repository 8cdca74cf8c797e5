"""The pipelined frequency loop (the next frequency's ACA on a second
stream while GMRES solves the current one) computes exactly what the
sequential loop computes: the kernels and their order on each operator are
the same, only the overlap differs."""

import sys

import numpy as np
import pytest

from synth import config_inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("store", ["c128", "c64"])
def test_pipeline_gives_identical_transients(store):
    import torch
    from paper_1212_3032_amd import ewbem as E
    d = config_inputs(2, sub=3)
    d["n_f"] = 32
    from synth import ramp_history
    d["history"] = ramp_history(32, d["period"], d["t_rise"])
    N = 3 * len(d["tri"])
    out = {}
    for pipe in (0, 1):
        c = E.Context(0)
        E.setup_from_inputs(c, d, op=dict(kind=E.OP_HMAT, leaf_size=64, eta_adm=1.0, aca_tol=1e-6,
                                          far_store=E.STORE_C64 if store == "c64" else E.STORE_C128),
                            solver=dict(tol=1e-8, guess=E.GUESS_SEM, pipeline=pipe))
        u = torch.zeros(d["n_f"] * N, dtype=torch.float64, device="cuda:0")
        st = c.solve_transient(u)
        st2 = c.solve_transient(u)  # a second pass over warm ACA lists
        out[pipe] = (u.cpu().numpy(), st, st2)
        c.close()
    (u0, a0, b0), (u1, a1, b1) = out[0], out[1]
    print(f"{store}: iterations {a0['iters_total']}/{b0['iters_total']} sequential, "
          f"{a1['iters_total']}/{b1['iters_total']} pipelined; max difference {np.abs(u0 - u1).max():.1e}",
          flush=True)
    sys.stdout.flush()
    assert (a0["iters_total"], b0["iters_total"]) == (a1["iters_total"], b1["iters_total"])
    assert a0["rank_sum"] == a1["rank_sum"] and b0["rank_sum"] == b1["rank_sum"]
    assert np.array_equal(u0, u1)
