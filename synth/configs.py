"""The five synthetic workloads, seeded.

``config_inputs(c)`` returns the mesh, material, time grid, load and method
options of workload ``c`` (1..5).  Seeds are ``CONFIG_SEED_BASE + c``.
"""

import numpy as np

from .mesh import icosphere, ellipsoid, merge_meshes, random_cavity_centres
from .loads import ramp_history, uniform_pressure, sh_pressure

CONFIG_SEED_BASE = 20121212

MATERIAL = dict(rho=1.0, mu=1.0, nu=0.25)


def _cavity(sub, period=8.0, n_f=32, sigma=None, t_rise=0.05, pressure=1.0):
    xyz, tri = icosphere(sub)
    return dict(
        xyz=xyz, tri=tri, exterior=1, material=dict(MATERIAL),
        period=period, n_f=n_f,
        sigma=(6.0 / period) if sigma is None else sigma,
        window=1,  # Hann
        pressure=uniform_pressure(len(tri), pressure),
        history=ramp_history(n_f, period, t_rise),
        t_rise=t_rise, radius=1.0,
    )


def config_inputs(c, sub=None):
    """Inputs of workload ``c``; ``sub`` overrides the icosphere level (used
    to run the same recipe at sizes the dense oracle can handle)."""
    rng = np.random.default_rng(CONFIG_SEED_BASE + int(c))
    if c == 1:
        d = _cavity(2 if sub is None else sub, n_f=32)
        d.update(name="sphere-sub2-dense", op=dict(kind=0),
                 solver=dict(tol=1e-8, guess=1, sem_k=3))
        return d
    if c == 2:
        d = _cavity(5 if sub is None else sub, n_f=128)
        d.update(name="sphere-sub5-hmat",
                 op=dict(kind=1, leaf_size=64, eta_adm=1.0, aca_tol=1e-5),
                 solver=dict(tol=1e-6, guess=1, sem_k=3))
        return d
    if c == 3:
        probs = []
        subs = [3, 3, 4, 4, 5, 5] + list(rng.choice([3, 4, 5], size=6))
        rng.shuffle(subs)
        for i in range(12):
            s = int(subs[i]) if sub is None else sub
            if i % 3 == 0:
                r = rng.uniform(0.5, 2.0)
                xyz, tri = icosphere(s, radius=r)
                axes = (r, r, r)
            else:
                axes = tuple(rng.uniform(0.5, 2.0, size=3))
                xyz, tri = ellipsoid(s, axes)
            amp = rng.uniform(0.5, 2.0)
            d = _cavity(0, n_f=128)
            d.update(xyz=xyz, tri=tri, pressure=uniform_pressure(len(tri), amp),
                     semi_axes=axes, name=f"cavity{i}-sub{s}",
                     op=dict(kind=1, leaf_size=64, eta_adm=1.0, aca_tol=1e-5,
                             far_store=1),
                     solver=dict(tol=1e-6, guess=1, sem_k=3))
            probs.append(d)
        return dict(name="12-cavities-batched", problems=probs)
    if c == 4:
        d = _cavity(5 if sub is None else sub, n_f=128)
        loads = []
        for _ in range(64):
            p, terms = sh_pressure(d["xyz"], d["tri"], rng)
            loads.append(p)
        d.update(name="sphere-sub5-64-sh-loads", loads=np.array(loads),
                 train=list(range(48)), held_out=list(range(48, 64)),
                 op=dict(kind=1, leaf_size=64, eta_adm=1.0, aca_tol=1e-5),
                 solver=dict(tol=1e-6, guess=1, sem_k=3))
        return d
    if c == 5:
        s = 5 if sub is None else sub
        centres = random_cavity_centres(rng, 12, 20.0, 2.5)
        xyz, tri = merge_meshes([icosphere(s, 1.0, cc) for cc in centres])
        d = _cavity(0, period=32.0, n_f=256, sigma=8.0 / 32.0)
        d.update(xyz=xyz, tri=tri, centres=centres, name="12-spheres-sub5",
                 op=dict(kind=1, leaf_size=64, eta_adm=1.0, aca_tol=1e-4,
                         far_store=1),
                 solver=dict(tol=1e-6, guess=1, sem_k=3))
        return d
    raise ValueError(f"unknown workload {c}")
