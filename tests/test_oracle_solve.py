"""End-to-end pin of the oracle's transient: the pressurised cavity.

The oracle's wall displacement through the whole pipeline (damped DFT,
dense solve per frequency, windowed de-damped inverse) is compared with
the same transform applied to the exact transfer function H(s_k): the
difference is the spatial discretisation error alone, which must shrink
under refinement.
"""

import numpy as np

from oracle import closed_form as CF, mft, solve
from synth import config_inputs


def _run(sub, n_f=16):
    d = config_inputs(1, sub=sub)
    from synth import ramp_history
    hist = ramp_history(n_f, d["period"], d["t_rise"])
    out = solve.transient(d["xyz"], d["tri"], d["material"], d["period"], n_f,
                          d["sigma"], d["window"], d["pressure"], hist)
    g = out["geom"]
    rh = g["cen"] / np.linalg.norm(g["cen"], axis=1, keepdims=True)
    ur = np.einsum("nek,ek->ne", out["u"].reshape(n_f, -1, 3), rh).mean(axis=1)
    spec = mft.load_spectrum(hist, d["period"], d["sigma"]) * CF.sphere_H(out["s"], 1.0, out["mat"])
    ref = mft.inverse(spec, d["period"], d["sigma"], d["window"])
    return np.linalg.norm(ur - ref) / np.linalg.norm(ref)


def test_transient_converges_to_transformed_closed_form():
    e0 = _run(0)
    e1 = _run(1)
    assert e1 < 0.1
    assert e1 < 0.7 * e0
