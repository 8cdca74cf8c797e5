"""CPU checks of the C-ABI library: it loads, exports every symbol the header
declares, validates its inputs, and its host-side cluster tree and block
partition are correct (no GPU needed: a host-only context)."""

import re
import os

import numpy as np
import pytest

from paper_1212_3032_amd import ewbem
from synth import icosphere, ellipsoid, config_inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    L = ewbem.lib()
    header = open(os.path.join(ROOT, "include", "ewbem.h")).read()
    declared = set(re.findall(r"\b(ewbem_[a-z_0-9]+)\s*\(", header))
    assert declared == set(ewbem.EXPORTED)
    for name in declared:
        assert hasattr(L, name), name


def test_defaults():
    o = ewbem.default_op_opts()
    assert (o.kind, o.leaf_size, o.eta_adm, o.aca_tol) == (ewbem.OP_HMAT, 64, 1.0, 1e-5)
    # the fields after the doubles sit where the C struct has them
    assert (o.far_store, o.self_order, o.aca_reuse, o.autotune) == (ewbem.STORE_C128, 24, 1, 1)
    # the warm start keeps every term it eliminates, down to the ACA tolerance
    assert (o.mv_mfma, o.ws_keep, o.ws_pivot_rel) == (1, 1, 0.0)
    s = ewbem.default_solver_opts()
    assert (s.tol, s.restart, s.guess, s.sem_k, s.pipeline) == (1e-6, 100, ewbem.GUESS_SEM, 3, 0)


def _ctx(sub=3, leaf=64, eta=1.0, kind=ewbem.OP_HMAT, axes=None):
    c = ewbem.Context(device=-1)
    xyz, tri = icosphere(sub) if axes is None else ellipsoid(sub, axes)
    c.set_mesh(xyz, tri)
    c.set_operator(kind=kind, leaf_size=leaf, eta_adm=eta)
    return c, xyz, tri


def _boxes(xyz, tri, perm, b, e):
    v = xyz[tri[perm[b:e]]].reshape(-1, 3)
    return v.min(axis=0), v.max(axis=0)


@pytest.mark.parametrize("sub,leaf,axes", [(3, 64, None), (3, 17, None), (4, 64, (1.5, 0.7, 1.0))])
def test_partition_covers_every_pair_once(sub, leaf, axes):
    c, xyz, tri = _ctx(sub, leaf, axes=axes)
    perm, near, far = c.partition()
    ne = len(tri)
    assert sorted(perm.tolist()) == list(range(ne))
    cover = np.zeros((ne, ne), np.int32)
    for r0, r1, c0, c1 in np.concatenate([near, far]):
        cover[r0:r1, c0:c1] += 1
    assert (cover == 1).all()
    info = c.info()
    assert info["max_leaf"] <= leaf
    # near blocks are leaf x leaf; the diagonal is near
    for r0, r1, c0, c1 in near:
        assert r1 - r0 <= leaf and c1 - c0 <= leaf
    # far blocks satisfy min(diam) <= eta dist on vertex bounding boxes
    for r0, r1, c0, c1 in far:
        lo1, hi1 = _boxes(xyz, tri, perm, r0, r1)
        lo2, hi2 = _boxes(xyz, tri, perm, c0, c1)
        d1, d2 = np.linalg.norm(hi1 - lo1), np.linalg.norm(hi2 - lo2)
        gap = np.maximum(0, np.maximum(lo1 - hi2, lo2 - hi1))
        assert min(d1, d2) <= 1.0 * np.linalg.norm(gap) + 1e-12
        assert np.linalg.norm(gap) > 0


def test_dense_kind_has_no_far_blocks():
    c, _, _ = _ctx(3, 64, kind=ewbem.OP_DENSE)
    info = c.info()
    assert info["n_far"] == 0
    assert info["near_entries"] == (3 * 1280) ** 2


def test_input_validation():
    c = ewbem.Context(device=-1)
    xyz, tri = icosphere(1)
    bad = tri.copy()
    bad[0, 0] = len(xyz)
    with pytest.raises(ewbem.EwbemError) as e:
        c.set_mesh(xyz, bad)
    assert e.value.status == ewbem.EINVAL
    deg = tri.copy()
    deg[0] = [0, 0, 1]
    with pytest.raises(ewbem.EwbemError):
        c.set_mesh(xyz, deg)
    with pytest.raises(ewbem.EwbemError) as e:
        c.set_material(1.0, 1.0, 0.5)
    assert e.value.status == ewbem.EINVAL
    with pytest.raises(ewbem.EwbemError):
        c.set_time(8.0, 31, 0.75)
    with pytest.raises(ewbem.EwbemError):
        c.set_operator(leaf_size=65)
    with pytest.raises(ewbem.EwbemError):
        c.set_operator(aca_reuse=2)
    with pytest.raises(ewbem.EwbemError):
        c.set_operator(ws_keep=2)
    with pytest.raises(ewbem.EwbemError):
        c.set_operator(ws_pivot_rel=1.0)
    c.set_operator(ws_keep=0, ws_pivot_rel=1e-6)
    c.set_mesh(xyz, tri)
    c.set_time(8.0, 16, 0.75)
    with pytest.raises(ewbem.EwbemError):
        c.set_load_pressure(np.full(len(tri), np.nan), np.ones(16))


def test_gpu_calls_refused_on_host_context():
    c = ewbem.Context(device=-1)
    d = config_inputs(1, sub=0)
    d["n_f"] = 4
    d["history"] = np.ones(4)
    c.set_mesh(d["xyz"], d["tri"])
    c.set_material(1, 1, 0.25)
    c.set_time(d["period"], 4, d["sigma"])
    c.set_load_pressure(d["pressure"], d["history"])
    with pytest.raises(ewbem.EwbemError) as e:
        c.load_spectrum()
    assert e.value.status == ewbem.ESTATE
    with pytest.raises(ewbem.EwbemError) as e:
        c.assemble(0)
    assert e.value.status == ewbem.ESTATE
    # the multi-load entry checks its arguments before it needs a device
    import ctypes
    L = ewbem.lib()
    p = np.ascontiguousarray(d["pressure"], dtype=np.float64)
    pp = p.ctypes.data_as(ctypes.c_void_p)
    assert L.ewbem_solve_transient_loads(c.h, 0, pp, 1, None, None, None) == ewbem.EINVAL
    assert L.ewbem_solve_transient_loads(c.h, 1, pp, 1, None, None, None) == ewbem.EINVAL
    assert L.ewbem_solve_transient_loads(c.h, 1, pp, 2, None, None, None) == ewbem.EINVAL
    # the incident-wave entry: arguments, then the context's load kind
    dq = np.array([1.0, 0.0, 0.0, 0.0, 0.0, 1.0])
    pd = dq.ctypes.data_as(ctypes.c_void_p)
    assert L.ewbem_solve_transient_incident_loads(c.h, 0, pd, pd, None, None, None) == ewbem.EINVAL
    assert L.ewbem_solve_transient_incident_loads(c.h, 1, pd, pd, None, None, None) == ewbem.EINVAL
    u_fake = ctypes.c_void_p(16)  # never touched: the pressure load is refused first
    assert L.ewbem_solve_transient_incident_loads(c.h, 1, pd, pd, u_fake, None, None) == ewbem.ESTATE


def _model_blob(n_dof, r, dims, rng, magic=b"EWBGUESS", version=2, rn=0, rk=0):
    import struct
    n_p = sum(dims[l + 1] * dims[l] + dims[l + 1] for l in range(len(dims) - 1))
    head = magic + struct.pack("<4i", version, n_dof, r, len(dims) - 1) + struct.pack(f"<{len(dims)}i", *dims)
    head += struct.pack("<3d", 0.99, 1e-2, 1e-4)
    p = rng.standard_normal(n_p).astype("<f4").tobytes()
    phi = (rng.standard_normal(n_dof * r) + 1j * rng.standard_normal(n_dof * r)).astype("<c16").tobytes()
    if version == 1:
        return head + p + phi
    nmap = max(0, rk - 3) * max(0, rn) * 4 * r
    tab = (rng.standard_normal(nmap) + 1j * rng.standard_normal(nmap)).astype("<c16").tobytes()
    return head + p + phi + struct.pack("<2i", rn, rk) + tab


def test_learned_model_format_on_host_context():
    c, xyz, tri = _ctx(2)
    N = 3 * len(tri)
    rng = np.random.default_rng(1)
    o = ewbem.default_train_opts()
    assert (o.n_modes, o.hidden, o.n_hidden, o.epochs, o.lr, o.power_iters, o.load_kind, o.seed,
            o.augment, o.unit_snapshots, o.lsq_map) == (64, 256, 3, 2000, 1e-3, 2, 0, 1, 4, 1, 1)
    with pytest.raises(ewbem.EwbemError) as e:
        c.guess_save()  # no model yet
    assert e.value.status == ewbem.ESTATE
    r = 5
    dims = [6 * r + 2, 16, 16, 2 * r]
    import struct
    # version 1 (no least-squares map) loads and is saved as version 2 with
    # an empty map
    v1 = _model_blob(N, r, dims, rng, version=1)
    c.guess_load(v1)
    assert c.guess_save() == v1[:8] + struct.pack("<i", 2) + v1[12:] + struct.pack("<2i", 0, 0)
    blob = _model_blob(N, r, dims, rng, rn=3, rk=7)
    c.guess_load(blob)
    assert c.guess_save() == blob  # a byte-exact round trip
    assert c.guess_basis() == r
    bad = [blob[:-1], blob + b"\0", b"X" + blob[1:], _model_blob(N + 3, r, dims, rng),
           _model_blob(N, r, [6 * r + 1, 16, 2 * r], rng), _model_blob(N, r, dims, rng, version=3),
           _model_blob(N, r, [6 * r + 2], rng), _model_blob(N, r, dims, rng, rn=3, rk=3),
           _model_blob(N, r, dims, rng, rn=0, rk=5), _model_blob(N, r, dims, rng, rn=-1, rk=5)]
    for b in bad:
        with pytest.raises(ewbem.EwbemError) as e:
            c.guess_load(b)
        assert e.value.status == ewbem.EINVAL
    nan = bytearray(blob)
    nan[len(blob) - 8:] = np.array([np.nan]).tobytes()
    with pytest.raises(ewbem.EwbemError):
        c.guess_load(bytes(nan))
    assert c.guess_save() == blob  # failed loads keep the model
    # the learned guess is a valid solver choice; 4 is not
    c.set_solver(guess=ewbem.GUESS_LEARNED)
    with pytest.raises(ewbem.EwbemError):
        c.set_solver(guess=4)
    # a new mesh drops the model
    c.set_mesh(xyz, tri)
    with pytest.raises(ewbem.EwbemError):
        c.guess_save()
    c.close()


def test_product_and_oracle_share_no_code():
    """The library and its binding never import the oracle, and the oracle
    never imports the library; synth/ (inputs only) is the one shared module."""
    import ast
    def imports(path):
        names = set()
        for root, _, files in os.walk(path):
            for f in files:
                if f.endswith(".py"):
                    tree = ast.parse(open(os.path.join(root, f)).read())
                    for node in ast.walk(tree):
                        if isinstance(node, ast.Import):
                            names.update(a.name.split(".")[0] for a in node.names)
                        elif isinstance(node, ast.ImportFrom) and node.module and node.level == 0:
                            names.add(node.module.split(".")[0])
        return names
    assert "oracle" not in imports(os.path.join(ROOT, "paper_1212_3032_amd"))
    assert "paper_1212_3032_amd" not in imports(os.path.join(ROOT, "oracle"))
    for root, _, files in os.walk(os.path.join(ROOT, "paper_1212_3032_amd", "csrc")):
        for f in files:
            assert "oracle" not in open(os.path.join(root, f), errors="ignore").read().lower(), f
    assert "paper_1212_3032_amd" not in imports(os.path.join(ROOT, "synth"))
    assert "oracle" not in imports(os.path.join(ROOT, "synth"))


def test_scene_full_size_partition_splits_large_admissible_pairs():
    """The twelve-cavity scene at level 5 (245,760 elements): admissible pairs
    of whole cavities exceed the far-block side limit of 16,384 elements and
    are split into admissible child pairs.  The blocks still cover every
    element pair exactly once (for every leaf, the column ranges of the
    blocks whose rows contain it tile 0..N_e), and no far block exceeds the
    limit on either side."""
    d = config_inputs(5, sub=5)
    c = ewbem.Context(device=-1)
    c.set_mesh(d["xyz"], d["tri"], exterior=True)
    c.set_operator(kind=ewbem.OP_HMAT, leaf_size=64, eta_adm=1.0, aca_tol=1e-4)
    perm, near, far = c.partition()
    ne = len(d["tri"])
    assert ne == 245760
    blocks = np.concatenate([near, far]).astype(np.int64)
    area = ((blocks[:, 1] - blocks[:, 0]) * (blocks[:, 3] - blocks[:, 2])).sum()
    assert area == ne * ne
    assert (far[:, 1] - far[:, 0]).max() <= 16384 and (far[:, 3] - far[:, 2]).max() <= 16384
    rows, inv = np.unique(blocks[:, :2], axis=0, return_inverse=True)
    cols = [blocks[inv.ravel() == g][:, 2:] for g in range(len(rows))]
    leaves = np.unique(near[:, :2], axis=0)
    assert leaves[0, 0] == 0 and leaves[-1, 1] == ne and (leaves[1:, 0] == leaves[:-1, 1]).all()
    for a, b in leaves:
        iv = np.concatenate([cols[g] for g in np.nonzero((rows[:, 0] <= a) & (rows[:, 1] >= b))[0]])
        iv = iv[np.argsort(iv[:, 0])]
        assert iv[0, 0] == 0 and iv[-1, 1] == ne and (iv[1:, 0] == iv[:-1, 1]).all()
