"""ctypes binding of libewbem.so (argument marshalling only).

Every computation runs in the HIP library; this module converts numpy arrays
and torch tensors to pointers, checks shapes, and turns status codes into
exceptions.  It fails loudly when the library has not been built.
"""

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libewbem.so")

OK, EINVAL, ENOMEM, EHIP, ENOCONV, ESTATE = 0, -1, -2, -3, -4, -5
OP_DENSE, OP_HMAT = 0, 1
STORE_C128, STORE_C64 = 0, 1
WINDOW_NONE, WINDOW_HANN, WINDOW_BLACKMAN = 0, 1, 2
PREC_NONE, PREC_ELEMENT, PREC_LEAF = 0, 1, 2
GUESS_ZERO, GUESS_SEM, GUESS_QUAD, GUESS_LEARNED = 0, 1, 2, 3

EXPORTED = [
    "ewbem_default_op_opts", "ewbem_default_solver_opts", "ewbem_create", "ewbem_destroy",
    "ewbem_last_error", "ewbem_set_mesh", "ewbem_set_material", "ewbem_set_time",
    "ewbem_set_load_traction", "ewbem_set_load_pressure", "ewbem_set_load_mixed",
    "ewbem_set_load_incident_s", "ewbem_set_load_incident_s_total",
    "ewbem_set_operator",
    "ewbem_set_solver", "ewbem_info", "ewbem_get_partition", "ewbem_load_spectrum",
    "ewbem_kernel_eval", "ewbem_assemble_dense", "ewbem_assemble", "ewbem_apply",
    "ewbem_apply_multi", "ewbem_get_rhs", "ewbem_solve_frequency", "ewbem_solve_transient", "ewbem_solve_transient_loads",
    "ewbem_solve_transient_incident_loads",
    "ewbem_batch_solve_transient", "ewbem_batch_solve_transient_lockstep",
    "ewbem_mft_inverse", "ewbem_default_train_opts", "ewbem_guess_train", "ewbem_guess_save",
    "ewbem_guess_load", "ewbem_guess_basis", "ewbem_mlp_eval", "ewbem_mlp_eval_noalloc", "ewbem_mlp_train",
]


class Z(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class OpOpts(C.Structure):
    _fields_ = [("kind", C.c_int32), ("leaf_size", C.c_int32), ("eta_adm", C.c_double),
                ("aca_tol", C.c_double), ("far_store", C.c_int32), ("self_order", C.c_int32),
                ("aca_reuse", C.c_int32), ("autotune", C.c_int32), ("aca_batch_mb", C.c_int32),
                ("mv_mfma", C.c_int32), ("ws_keep", C.c_int32), ("ws_pivot_rel", C.c_double)]


class SolverOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int32), ("maxit", C.c_int32),
                ("precond", C.c_int32), ("guess", C.c_int32), ("sem_k", C.c_int32),
                ("pipeline", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_solves", C.c_int32), ("iters_total", C.c_int32), ("iters_max", C.c_int32),
                ("matvecs", C.c_int32), ("resid_max", C.c_double), ("guess_resid_sum", C.c_double),
                ("t_assemble_ms", C.c_double), ("t_guess_ms", C.c_double),
                ("t_gmres_ms", C.c_double), ("t_post_ms", C.c_double), ("t_matvec_ms", C.c_double),
                ("matvec_bytes", C.c_double), ("stored_bytes", C.c_double),
                ("n_near", C.c_int64), ("n_far", C.c_int64), ("rank_sum", C.c_int64),
                ("rank_max", C.c_int64), ("t_aca_ms", C.c_double), ("t_near_ms", C.c_double),
                ("t_rhs_ms", C.c_double), ("matvec_bytes_total", C.c_double),
                ("matvecs_timed", C.c_int32), ("pad0", C.c_int32),
                ("aca_warm_blocks", C.c_int64), ("aca_cold_blocks", C.c_int64),
                ("guess_learned", C.c_int64), ("pod_energy", C.c_double),
                ("train_loss_first", C.c_double), ("train_loss_last", C.c_double),
                ("aca_core_blocks", C.c_int64 * 7), ("aca_warm_pivots", C.c_int64),
                ("aca_warm_kept", C.c_int64), ("aca_retries", C.c_int64),
                ("aca_steps", C.c_int64), ("aca_step_blocks", C.c_int64), ("aca_step_first", C.c_int64)]

    def as_dict(self):
        return {f: (list(getattr(self, f)) if f == "aca_core_blocks" else getattr(self, f))
                for f, _ in self._fields_}


class TrainOpts(C.Structure):
    _fields_ = [("n_modes", C.c_int32), ("hidden", C.c_int32), ("n_hidden", C.c_int32),
                ("epochs", C.c_int32), ("lr", C.c_double), ("power_iters", C.c_int32),
                ("load_kind", C.c_int32), ("seed", C.c_uint64), ("augment", C.c_int32),
                ("unit_snapshots", C.c_int32), ("lsq_map", C.c_int32), ("pad", C.c_int32),
                ("lsq_reg", C.c_double)]


class Info(C.Structure):
    _fields_ = [("n_elements", C.c_int64), ("n_dof", C.c_int64), ("n_clusters", C.c_int64),
                ("n_leaves", C.c_int64), ("n_near", C.c_int64), ("n_far", C.c_int64),
                ("near_entries", C.c_int64), ("max_leaf", C.c_int32), ("min_leaf", C.c_int32),
                ("mv_cols", C.c_int32), ("mv_task_div", C.c_int32), ("mv_tuned", C.c_int32),
                ("mv_tune_cached", C.c_int32), ("mv_tune_best_ms", C.c_double), ("mv_tune_default_ms", C.c_double),
                ("lib_device_bytes", C.c_int64), ("far_work_bytes", C.c_int64),
                ("aca_scratch_bytes", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    """Load libewbem.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "or python paper_1212_3032_amd/build.py")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "ewbem_default_op_opts": (None, [C.POINTER(OpOpts)]),
        "ewbem_default_solver_opts": (None, [C.POINTER(SolverOpts)]),
        "ewbem_create": (C.c_int, [C.POINTER(P), I32, P]),
        "ewbem_destroy": (None, [P]),
        "ewbem_last_error": (C.c_char_p, [P]),
        "ewbem_set_mesh": (C.c_int, [P, I64, P, I64, P, I32]),
        "ewbem_set_material": (C.c_int, [P, D, D, D]),
        "ewbem_set_time": (C.c_int, [P, D, I32, D, I32]),
        "ewbem_set_load_traction": (C.c_int, [P, P, P]),
        "ewbem_set_load_pressure": (C.c_int, [P, P, P]),
        "ewbem_set_load_mixed": (C.c_int, [P, P, P, P]),
        "ewbem_set_load_incident_s": (C.c_int, [P, P, P, D, D]),
        "ewbem_set_load_incident_s_total": (C.c_int, [P, P, P, D, D]),
        "ewbem_set_operator": (C.c_int, [P, C.POINTER(OpOpts)]),
        "ewbem_set_solver": (C.c_int, [P, C.POINTER(SolverOpts)]),
        "ewbem_info": (C.c_int, [P, C.POINTER(Info)]),
        "ewbem_get_partition": (C.c_int, [P, P, P, P]),
        "ewbem_load_spectrum": (C.c_int, [P, P]),
        "ewbem_kernel_eval": (C.c_int, [P, Z, I64, P, P, P, P, P]),
        "ewbem_assemble_dense": (C.c_int, [P, Z, P, P]),
        "ewbem_assemble": (C.c_int, [P, I32, C.POINTER(Stats)]),
        "ewbem_apply": (C.c_int, [P, P, P]),
        "ewbem_apply_multi": (C.c_int, [P, P, I32, P]),
        "ewbem_get_rhs": (C.c_int, [P, P]),
        "ewbem_solve_frequency": (C.c_int, [P, I32, P, P, C.POINTER(Stats)]),
        "ewbem_solve_transient": (C.c_int, [P, P, P, C.POINTER(Stats)]),
        "ewbem_solve_transient_loads": (C.c_int, [P, I32, P, I32, P, P, C.POINTER(Stats)]),
        "ewbem_solve_transient_incident_loads": (C.c_int, [P, I32, P, P, P, P, C.POINTER(Stats)]),
        "ewbem_batch_solve_transient": (C.c_int, [P, I32, P, C.POINTER(Stats), I32]),
        "ewbem_batch_solve_transient_lockstep": (C.c_int, [P, I32, P, C.POINTER(Stats), I32]),
        "ewbem_mft_inverse": (C.c_int, [P, P, P]),
        "ewbem_default_train_opts": (None, [C.POINTER(TrainOpts)]),
        "ewbem_guess_train": (C.c_int, [P, I32, P, C.POINTER(TrainOpts), C.POINTER(Stats)]),
        "ewbem_guess_save": (C.c_int, [P, P, C.POINTER(C.c_size_t)]),
        "ewbem_guess_load": (C.c_int, [P, P, C.c_size_t]),
        "ewbem_guess_basis": (C.c_int, [P, C.POINTER(I32), P]),
        "ewbem_mlp_eval": (C.c_int, [P, I32, P, P, I64, P, P, P, P, C.POINTER(D)]),
        "ewbem_mlp_eval_noalloc": (C.c_int, [P, I32, P, P, I64, P, P, P, P, C.POINTER(D)]),
        "ewbem_mlp_train": (C.c_int, [P, I32, P, P, I64, P, P, I32, D, C.POINTER(D), C.POINTER(D)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


class EwbemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ewbem status {status}: {msg}")
        self.status = status


def default_op_opts(**kw):
    o = OpOpts()
    lib().ewbem_default_op_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def default_solver_opts(**kw):
    o = SolverOpts()
    lib().ewbem_default_solver_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def default_train_opts(**kw):
    o = TrainOpts()
    lib().ewbem_default_train_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


def _dev_ptr(t, dtype_name, numel=None):
    """Device pointer of a contiguous CUDA (HIP) torch tensor."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a GPU torch tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if str(t.dtype) != dtype_name:
        raise TypeError(f"expected {dtype_name}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


class Context:
    """One ewbem context.  ``device`` = -1 makes a host-only context."""

    def __init__(self, device=0, stream=None):
        self._L = lib()
        h = C.c_void_p()
        if device >= 0 and stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        st = self._L.ewbem_create(C.byref(h), int(device), C.c_void_p(stream or 0))
        if st != OK:
            raise EwbemError(st, "could not create context")
        self.h = h
        self.device = device
        self.nt = 0
        self.n_f = 0

    def close(self):
        if getattr(self, "h", None):
            self._L.ewbem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st):
        if st != OK:
            raise EwbemError(st, self._L.ewbem_last_error(self.h).decode())
        return st

    # ---- setup
    def set_mesh(self, xyz, tri, exterior=True):
        xyz, px = _host(xyz, np.float64)
        tri, pt = _host(tri, np.int32)
        self._check(self._L.ewbem_set_mesh(self.h, len(xyz), px, len(tri), pt, int(bool(exterior))))
        self.nt = len(tri)

    def set_material(self, rho, mu, nu):
        self._check(self._L.ewbem_set_material(self.h, rho, mu, nu))

    def set_time(self, period, n_f, sigma, window=WINDOW_HANN):
        self._check(self._L.ewbem_set_time(self.h, period, int(n_f), sigma, int(window)))
        self.n_f = int(n_f)

    def set_load_pressure(self, p, history):
        p, pp = _host(p, np.float64)
        h, ph = _host(history, np.float64)
        if p.shape != (self.nt,) or h.shape != (self.n_f,):
            raise ValueError("pressure must have nt values and history n_f samples")
        self._check(self._L.ewbem_set_load_pressure(self.h, pp, ph))

    def set_load_traction(self, t0, history):
        t0, pt = _host(t0, np.float64)
        h, ph = _host(history, np.float64)
        if t0.size != 3 * self.nt or h.shape != (self.n_f,):
            raise ValueError("traction must have 3 nt values and history n_f samples")
        self._check(self._L.ewbem_set_load_traction(self.h, pt, ph))

    def set_load_mixed(self, bc, values, history):
        """bc: 0 = given traction, 1 = given (zero) displacement per element;
        values: nt x 3 given tractions (zero rows for bc 1)."""
        bc, pb = _host(bc, np.int32)
        v, pv = _host(values, np.float64)
        h, ph = _host(history, np.float64)
        if bc.shape != (self.nt,) or v.size != 3 * self.nt or h.shape != (self.n_f,):
            raise ValueError("bc must have nt entries, values 3 nt, history n_f")
        self._check(self._L.ewbem_set_load_mixed(self.h, pb, pv, ph))

    def set_load_incident_s(self, direction, polarisation, ricker_fc, t0, total=False):
        """Plane S-wave u_inc = pol f(t - dir.x / c_s), f a Ricker wavelet of
        centre frequency ricker_fc peaking at t0; outputs are the scattered
        displacement, or with ``total`` (the total-field formulation, whose
        right-hand side is u_inc itself) the total displacement."""
        d, pd = _host(direction, np.float64)
        q, pq = _host(polarisation, np.float64)
        if d.shape != (3,) or q.shape != (3,):
            raise ValueError("direction and polarisation must have 3 entries")
        fn = self._L.ewbem_set_load_incident_s_total if total else self._L.ewbem_set_load_incident_s
        self._check(fn(self.h, pd, pq, float(ricker_fc), float(t0)))

    def set_operator(self, **kw):
        o = default_op_opts(**kw)
        self._check(self._L.ewbem_set_operator(self.h, C.byref(o)))

    def set_solver(self, **kw):
        o = default_solver_opts(**kw)
        self._check(self._L.ewbem_set_solver(self.h, C.byref(o)))

    def info(self):
        i = Info()
        self._check(self._L.ewbem_info(self.h, C.byref(i)))
        return i.as_dict()

    def partition(self):
        inf = self.info()
        perm = np.zeros(self.nt, np.int32)
        near = np.zeros((inf["n_near"], 4), np.int32)
        far = np.zeros((max(inf["n_far"], 0), 4), np.int32)
        self._check(self._L.ewbem_get_partition(
            self.h, perm.ctypes.data_as(C.c_void_p), near.ctypes.data_as(C.c_void_p),
            far.ctypes.data_as(C.c_void_p)))
        return perm, near, far

    # ---- compute (device tensors)
    def load_spectrum(self):
        out = np.zeros(self.n_f // 2 + 1, np.complex128)
        self._check(self._L.ewbem_load_spectrum(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    def kernel_eval(self, s, x, y, nrm, U=None, T=None):
        n = x.shape[0]
        px = _dev_ptr(x, "torch.float64", 3 * n)
        py = _dev_ptr(y, "torch.float64", 3 * n)
        pn = _dev_ptr(nrm, "torch.float64", 3 * n)
        pU = _dev_ptr(U, "torch.complex128", 9 * n) if U is not None else None
        pT = _dev_ptr(T, "torch.complex128", 9 * n) if T is not None else None
        self._check(self._L.ewbem_kernel_eval(self.h, Z(s.real, s.imag), n, px, py, pn, pU, pT))

    def assemble_dense(self, s, T=None, U=None):
        N = 3 * self.nt
        pT = _dev_ptr(T, "torch.complex128", N * N) if T is not None else None
        pU = _dev_ptr(U, "torch.complex128", N * N) if U is not None else None
        self._check(self._L.ewbem_assemble_dense(self.h, Z(complex(s).real, complex(s).imag), pT, pU))

    def assemble(self, k):
        st = Stats()
        self._check(self._L.ewbem_assemble(self.h, int(k), C.byref(st)))
        return st.as_dict()

    def apply(self, x, y):
        N = 3 * self.nt
        self._check(self._L.ewbem_apply(self.h, _dev_ptr(x, "torch.complex128", N),
                                        _dev_ptr(y, "torch.complex128", N)))

    def apply_multi(self, X, Y):
        """Y[j] = A X[j] for the rows of X (nrhs x N complex128, nrhs <= 8)."""
        N = 3 * self.nt
        nrhs = int(X.shape[0])
        if tuple(X.shape) != (nrhs, N) or tuple(Y.shape) != (nrhs, N):
            raise ValueError("apply_multi: X and Y must be nrhs x N")
        self._check(self._L.ewbem_apply_multi(self.h, _dev_ptr(X, "torch.complex128", nrhs * N), nrhs,
                                              _dev_ptr(Y, "torch.complex128", nrhs * N)))

    def get_rhs(self, b):
        self._check(self._L.ewbem_get_rhs(self.h, _dev_ptr(b, "torch.complex128", 3 * self.nt)))

    def solve_frequency(self, k, a, x0=None, allow_noconv=False):
        N = 3 * self.nt
        st = Stats()
        px0 = _dev_ptr(x0, "torch.complex128", N) if x0 is not None else None
        rc = self._L.ewbem_solve_frequency(self.h, int(k), px0, _dev_ptr(a, "torch.complex128", N),
                                           C.byref(st))
        if not (allow_noconv and rc == ENOCONV):
            self._check(rc)
        return st.as_dict()

    def solve_transient(self, u, spec=None, allow_noconv=False):
        N = 3 * self.nt
        st = Stats()
        ps = _dev_ptr(spec, "torch.complex128", (self.n_f // 2 + 1) * N) if spec is not None else None
        rc = self._L.ewbem_solve_transient(self.h, _dev_ptr(u, "torch.float64", self.n_f * N), ps,
                                           C.byref(st))
        if not (allow_noconv and rc == ENOCONV):
            self._check(rc)
        return st.as_dict()

    def solve_transient_loads(self, loads, u, spec=None, pressures=False, allow_noconv=False):
        """Several loads with the current load's history on shared per-
        frequency operators: loads n_loads x nt x 3 tractions (or n_loads x
        nt pressures), u a device float64 tensor of n_loads x n_f x N."""
        N = 3 * self.nt
        per = self.nt if pressures else 3 * self.nt
        a, pa = _host(loads, np.float64)
        if a.size % per != 0 or a.size == 0:
            raise ValueError(f"loads must hold n_loads x {per} values")
        n = a.size // per
        ps = _dev_ptr(spec, "torch.complex128", n * (self.n_f // 2 + 1) * N) if spec is not None else None
        st = Stats()
        rc = self._L.ewbem_solve_transient_loads(self.h, n, pa, 1 if pressures else 0,
                                                 _dev_ptr(u, "torch.float64", n * self.n_f * N), ps, C.byref(st))
        if not (allow_noconv and rc == ENOCONV):
            self._check(rc)
        return st.as_dict()

    def solve_transient_incident_loads(self, dirs, pols, u, spec=None, allow_noconv=False):
        """Several incident plane S-waves (n x 3 directions and polarisations)
        with the current incident wave's wavelet, through one frequency
        loop: u a device float64 tensor of n x n_f x N."""
        N = 3 * self.nt
        a, pa = _host(dirs, np.float64)
        b, pb = _host(pols, np.float64)
        if a.size % 3 != 0 or a.size == 0 or b.size != a.size:
            raise ValueError("dirs and pols must both hold n x 3 values")
        n = a.size // 3
        ps = _dev_ptr(spec, "torch.complex128", n * (self.n_f // 2 + 1) * N) if spec is not None else None
        st = Stats()
        rc = self._L.ewbem_solve_transient_incident_loads(self.h, n, pa, pb,
                                                          _dev_ptr(u, "torch.float64", n * self.n_f * N), ps,
                                                          C.byref(st))
        if not (allow_noconv and rc == ENOCONV):
            self._check(rc)
        return st.as_dict()

    def guess_train(self, loads, pressures=False, allow_noconv=False, **kw):
        """Train the learned guess on several loads (n_cases x nt x 3
        tractions, or n_cases x nt pressures); keyword options as in
        TrainOpts.  Returns the stats (training solves, pod_energy, losses)."""
        o = default_train_opts(load_kind=1 if pressures else 0, **kw)
        per = self.nt if pressures else 3 * self.nt
        a, pa = _host(loads, np.float64)
        if a.size % per != 0 or a.size == 0:
            raise ValueError(f"loads must hold n_cases x {per} values")
        st = Stats()
        rc = self._L.ewbem_guess_train(self.h, a.size // per, pa, C.byref(o), C.byref(st))
        if not (allow_noconv and rc == ENOCONV):
            self._check(rc)
        return st.as_dict()

    def guess_save(self):
        n = C.c_size_t(0)
        self._check(self._L.ewbem_guess_save(self.h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(self._L.ewbem_guess_save(self.h, buf, C.byref(n)))
        return buf.raw[:n.value]

    def guess_load(self, data):
        data = bytes(data)
        buf = C.create_string_buffer(data, len(data))
        self._check(self._L.ewbem_guess_load(self.h, buf, len(data)))

    def guess_basis(self, phi=None):
        """Basis size r; with phi (device complex128 tensor of N x r entries,
        column-major, i.e. shape (r, N)) also the basis."""
        r = C.c_int32(0)
        self._check(self._L.ewbem_guess_basis(self.h, C.byref(r), None))
        if phi is not None:
            self._check(self._L.ewbem_guess_basis(
                self.h, C.byref(r), _dev_ptr(phi, "torch.complex128", 3 * self.nt * r.value)))
        return r.value

    def mlp_eval(self, dims, params, x, y, target=None, grad=None, noalloc=False):
        """The network's kernels on device float32 tensors; returns the loss
        (0 without a target).  noalloc: through ewbem_mlp_eval_noalloc (no
        device allocation; its buffers in the library's static scratch)."""
        d, pd = _host(dims, np.int32)
        L = d.size - 1
        batch = x.numel() // int(d[0]) if int(d[0]) > 0 else 0
        np_ = sum(int(d[l + 1]) * int(d[l]) + int(d[l + 1]) for l in range(L))
        loss = C.c_double(0.0)
        fn = self._L.ewbem_mlp_eval_noalloc if noalloc else self._L.ewbem_mlp_eval
        self._check(fn(
            self.h, L, pd, _dev_ptr(params, "torch.float32", np_), batch,
            _dev_ptr(x, "torch.float32", batch * int(d[0])) if batch else None,
            _dev_ptr(target, "torch.float32", batch * int(d[-1])) if target is not None else None,
            _dev_ptr(y, "torch.float32", batch * int(d[-1])) if batch else None,
            _dev_ptr(grad, "torch.float32", np_) if grad is not None else None, C.byref(loss)))
        return loss.value

    def mlp_train(self, dims, params, x, target, epochs, lr):
        """Full-batch Adam steps on device float32 tensors (params in place);
        returns (first loss, last loss)."""
        d, pd = _host(dims, np.int32)
        L = d.size - 1
        batch = x.numel() // int(d[0])
        np_ = sum(int(d[l + 1]) * int(d[l]) + int(d[l + 1]) for l in range(L))
        l0, l1 = C.c_double(0.0), C.c_double(0.0)
        self._check(self._L.ewbem_mlp_train(
            self.h, L, pd, _dev_ptr(params, "torch.float32", np_), batch,
            _dev_ptr(x, "torch.float32", batch * int(d[0])),
            _dev_ptr(target, "torch.float32", batch * int(d[-1])), int(epochs), float(lr),
            C.byref(l0), C.byref(l1)))
        return l0.value, l1.value

    def mft_inverse(self, spec, u):
        N = 3 * self.nt
        self._check(self._L.ewbem_mft_inverse(
            self.h, _dev_ptr(spec, "torch.complex128", (self.n_f // 2 + 1) * N),
            _dev_ptr(u, "torch.float64", self.n_f * N)))


def batch_solve_transient(ctxs, outs, per_launch=16, allow_noconv=False, lockstep=False):
    """Solve the transients of several contexts (distinct, ideally each on its
    own stream) concurrently; outs[i] is context i's n_f x 3 nt float64
    device tensor.  lockstep: in groups of per_launch over the frequency
    index, one concatenated matvec per Arnoldi step of the group
    (ewbem_batch_solve_transient_lockstep).  Returns the aggregated stats."""
    if len(ctxs) != len(outs):
        raise ValueError("one output per context")
    n = len(ctxs)
    hs = (C.c_void_p * max(n, 1))(*[c.h.value for c in ctxs])
    us = (C.c_void_p * max(n, 1))(*[_dev_ptr(u, "torch.float64", c.n_f * 3 * c.nt).value
                                    for c, u in zip(ctxs, outs)])
    st = Stats()
    fn = lib().ewbem_batch_solve_transient_lockstep if lockstep else lib().ewbem_batch_solve_transient
    rc = fn(hs, n, us, C.byref(st), int(per_launch))
    if rc != OK and not (allow_noconv and rc == ENOCONV):
        raise EwbemError(rc, "batch transient solve failed: " + "; ".join(
            (lib().ewbem_last_error(c.h) or b"").decode() for c in ctxs))
    return st.as_dict()


def setup_from_inputs(ctx, d, op=None, solver=None):
    """Configure a context from a ``synth.config_inputs`` dictionary."""
    ctx.set_mesh(d["xyz"], d["tri"], exterior=bool(d.get("exterior", 1)))
    m = d["material"]
    ctx.set_material(m["rho"], m["mu"], m["nu"])
    ctx.set_time(d["period"], d["n_f"], d["sigma"], d["window"])
    ctx.set_load_pressure(d["pressure"], d["history"])
    ctx.set_operator(**(op if op is not None else d.get("op", {})))
    ctx.set_solver(**(solver if solver is not None else d.get("solver", {})))
    return ctx
