"""ctypes binding of libsdg.so (the C ABI declared in include/sdg.h).

Argument marshalling only: every function forwards to the library entry
point of the same name.  Device arrays are torch tensors on the GPU (their
data_ptr() is passed); host arrays are numpy arrays.  The library is
required: importing this module on a machine where it is not built raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libsdg.so")

NAVIER, NEUMANN, DIRICHLET = 0, 1, 2
FP64, FP32, BF16 = 0, 1, 2
OK, ERR_INVALID, ERR_NOMEM, ERR_DEVICE, ERR_UNSUPPORTED = 0, -1, -2, -3, -4
NOT_CONVERGED, BREAKDOWN, FLOOR = 1, 2, 3


class sdg_mesh(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("lx", ctypes.c_double),
                ("ly", ctypes.c_double), ("k", ctypes.c_int32), ("bc", ctypes.c_int32 * 4)]


class sdg_options(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("inner_rtol", ctypes.c_double),
                ("max_it", ctypes.c_int32), ("inner_max_it", ctypes.c_int32),
                ("restart", ctypes.c_int32), ("smooth_dg", ctypes.c_int32),
                ("smooth_h", ctypes.c_int32), ("coarsest_n", ctypes.c_int32),
                ("eig_steps", ctypes.c_int32), ("cheb_lo", ctypes.c_double),
                ("cheb_hi", ctypes.c_double), ("prec_smoother", ctypes.c_int32),
                ("prec_apply", ctypes.c_int32), ("viscous_krylov", ctypes.c_int32),
                ("dedup", ctypes.c_int32), ("seed", ctypes.c_uint64), ("graphs", ctypes.c_int32),
                ("refine", ctypes.c_int32), ("outer_krylov", ctypes.c_int32), ("coarse_space", ctypes.c_int32)]


class sdg_stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("outer_its", ctypes.c_int32),
                ("inner_its_total", ctypes.c_int32), ("inner_its_max", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("setup_ms", ctypes.c_double),
                ("solve_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class sdg_server_config(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("bypass", ctypes.c_int32),
                ("combine", ctypes.c_int32), ("mem_budget", ctypes.c_size_t)]


class sdg_req_info(ctypes.Structure):
    _fields_ = [("submit_ms", ctypes.c_double), ("start_ms", ctypes.c_double),
                ("end_ms", ctypes.c_double), ("batch", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("bytes", ctypes.c_size_t)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad_"}


VISCOUS, STOKES = 0, 1
P = ctypes.c_void_p
PP = ctypes.POINTER(ctypes.c_void_p)
I = ctypes.c_int
MESH = ctypes.POINTER(sdg_mesh)
OPTS = ctypes.POINTER(sdg_options)
STATS = ctypes.POINTER(sdg_stats)

# name -> (restype, argtypes); every symbol declared in include/sdg.h
PROTOTYPES = {
    "sdg_create": (I, [I, ctypes.c_size_t, PP]),
    "sdg_destroy": (None, [P]),
    "sdg_last_error": (ctypes.c_char_p, []),
    "sdg_options_default": (None, [OPTS]),
    "sdg_required_bytes": (ctypes.c_size_t, [MESH, OPTS, I]),
    "sdg_problem_create": (I, [P, MESH, OPTS, P, P, PP]),
    "sdg_problem_create_batch": (I, [P, MESH, OPTS, I, P, P, PP]),
    "sdg_problem_batch": (I, [P, ctypes.POINTER(ctypes.c_int)]),
    "sdg_problem_smoother_precision": (I, [P, ctypes.POINTER(ctypes.c_int)]),
    "sdg_required_bytes_batch": (ctypes.c_size_t, [MESH, OPTS, I, I]),
    "sdg_problem_destroy": (None, [P]),
    "sdg_problem_levels": (I, [P, ctypes.POINTER(ctypes.c_int)]),
    "sdg_get_bounds": (I, [P, ctypes.POINTER(ctypes.c_double)]),
    "sdg_set_bounds": (I, [P, ctypes.POINTER(ctypes.c_double)]),
    "sdg_eig_estimate": (I, [P, I, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "sdg_apply_viscous": (I, [P, P, P]),
    "sdg_residual_viscous": (I, [P, P, P, P]),
    "sdg_apply_viscous_f32": (I, [P, P, P]),
    "sdg_apply_div": (I, [P, P, P]),
    "sdg_apply_grad": (I, [P, P, P]),
    "sdg_apply_blockjacobi": (I, [P, P, P]),
    "sdg_get_blocks": (I, [P, P]),
    "sdg_get_blocks_noalloc": (I, [P, P]),
    "sdg_p_restrict": (I, [P, P, P]),
    "sdg_p_prolong_add": (I, [P, P, P]),
    "sdg_get_coarse_stencil": (I, [P, I, P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "sdg_vcycle": (I, [P, P, P]),
    "sdg_assemble_rhs": (I, [P, P, P, P, P]),
    "sdg_solve_viscous_dev": (I, [P, P, P, P, STATS]),
    "sdg_solve_stokes_dev": (I, [P, P, P, P, P, STATS]),
    "sdg_solve_viscous_ext_dev": (I, [P, P, P, P, P, STATS]),
    "sdg_solve_stokes_ext_dev": (I, [P, P, P, P, P, P, P, STATS]),
    "sdg_residual_ext": (I, [P, I, P, P, P, P]),
    "sdg_abs_apply": (I, [P, I, P, P]),
    "sdg_solve_viscous_batch": (I, [P, I, MESH, OPTS, P, P, P, P, STATS]),
    "sdg_solve_viscous": (I, [P, MESH, OPTS, P, P, P, P, STATS]),
    "sdg_solve_stokes": (I, [P, MESH, OPTS, P, P, P, P, P, STATS]),
    "sdg_uniform_pm1": (I, [P, ctypes.c_uint64, ctypes.c_int64, P, P]),
    "sdg_tile_variants": (I, [I, ctypes.POINTER(I)]),
    "sdg_tile_shape": (I, [I, I, ctypes.POINTER(I), ctypes.POINTER(I)]),
    "sdg_get_tile": (I, [P, I, I, ctypes.POINTER(I)]),
    "sdg_set_tile": (I, [P, I, I, I]),
    "sdg_autotune": (I, [P, I, ctypes.POINTER(I), ctypes.POINTER(ctypes.c_double)]),
    "sdg_server_config_default": (None, [ctypes.POINTER(sdg_server_config)]),
    "sdg_server_create": (I, [P, ctypes.POINTER(sdg_server_config), PP]),
    "sdg_server_destroy": (None, [P]),
    "sdg_submit": (I, [P, MESH, OPTS, I, P, P, P, PP]),
    "sdg_poll": (I, [P, ctypes.POINTER(I)]),
    "sdg_wait": (I, [P, P, P, STATS, ctypes.POINTER(sdg_req_info)]),
    "sdg_req_free": (None, [P]),
    "sdg_server_stats": (I, [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_size_t),
                             ctypes.POINTER(I), ctypes.POINTER(ctypes.c_size_t)]),
    "sdg_admission_simulate": (I, [I, P, P, P, I, ctypes.c_size_t, I, P]),
    "sdg_server_launch_stats": (I, [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(I), ctypes.POINTER(ctypes.c_int64)]),
    "sdg_trace_enable": (I, [P, I]),
    "sdg_trace_read": (I, [P, I, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(ctypes.c_double)]),
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is not built; run paper_1607_03777_amd.build.build()")
        L = ctypes.CDLL(LIBPATH)
        for name, (res, args) in PROTOTYPES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class SDGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sdg error {code}: {msg}")
        self.code = code


def check(rc):
    if rc < 0:
        raise SDGError(rc, lib().sdg_last_error().decode())
    return rc


def ptr(t):
    """Device or host pointer of a torch tensor / numpy array (None -> NULL)."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        assert t.flags["C_CONTIGUOUS"]
        return t.ctypes.data
    assert t.is_contiguous()
    return t.data_ptr()


def make_mesh(nx, ny, k, bc=(NAVIER,) * 4, lx=1.0, ly=1.0):
    m = sdg_mesh()
    m.nx, m.ny, m.lx, m.ly, m.k = nx, ny, lx, ly, k
    for i in range(4):
        m.bc[i] = bc[i]
    return m


def make_options(**kw):
    o = sdg_options()
    lib().sdg_options_default(ctypes.byref(o))
    for key, v in kw.items():
        if not hasattr(o, key):
            raise KeyError(key)
        setattr(o, key, v)
    return o


def current_stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


# ---- thin wrappers with the C names ---------------------------------------
def sdg_create(device=0, mem_budget=0):
    out = ctypes.c_void_p()
    check(lib().sdg_create(device, mem_budget, ctypes.byref(out)))
    return out


def sdg_destroy(ctx):
    lib().sdg_destroy(ctx)


def sdg_required_bytes(mesh, opts, stokes):
    return lib().sdg_required_bytes(ctypes.byref(mesh), ctypes.byref(opts), int(stokes))


def sdg_problem_create(ctx, mesh, opts, eta_dev, stream=None):
    out = ctypes.c_void_p()
    check(lib().sdg_problem_create(ctx, ctypes.byref(mesh), ctypes.byref(opts), ptr(eta_dev),
                                   stream, ctypes.byref(out)))
    return out


def sdg_problem_create_batch(ctx, mesh, opts, nbatch, eta_dev, stream=None):
    out = ctypes.c_void_p()
    check(lib().sdg_problem_create_batch(ctx, ctypes.byref(mesh), ctypes.byref(opts), int(nbatch),
                                         ptr(eta_dev), stream, ctypes.byref(out)))
    return out


def sdg_problem_batch(prob):
    n = ctypes.c_int()
    check(lib().sdg_problem_batch(prob, ctypes.byref(n)))
    return n.value


def sdg_problem_smoother_precision(prob):
    n = ctypes.c_int()
    check(lib().sdg_problem_smoother_precision(prob, ctypes.byref(n)))
    return n.value


def sdg_required_bytes_batch(mesh, opts, stokes, nbatch):
    return lib().sdg_required_bytes_batch(ctypes.byref(mesh), ctypes.byref(opts), int(stokes), int(nbatch))


def sdg_problem_destroy(prob):
    lib().sdg_problem_destroy(prob)


def sdg_problem_levels(prob):
    n = ctypes.c_int()
    check(lib().sdg_problem_levels(prob, ctypes.byref(n)))
    return n.value


def sdg_get_bounds(prob):
    """[nbatch][nlevels][2] array (a batch of one is returned as [nlevels][2])."""
    n = sdg_problem_levels(prob)
    nb = sdg_problem_batch(prob)
    b = np.zeros((nb, n, 2))
    check(lib().sdg_get_bounds(prob, b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return b[0] if nb == 1 else b


def sdg_set_bounds(prob, bounds):
    n = sdg_problem_levels(prob)
    nb = sdg_problem_batch(prob)
    b = np.ascontiguousarray(np.broadcast_to(np.asarray(bounds, dtype=np.float64), (nb, n, 2)))
    check(lib().sdg_set_bounds(prob, b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))


def sdg_eig_estimate(prob, level, steps=10):
    """Returns (lambda[nbatch], H[nbatch][steps+1][steps])."""
    nb = sdg_problem_batch(prob)
    lam = np.zeros(nb)
    H = np.zeros((nb, steps, steps + 1))
    check(lib().sdg_eig_estimate(prob, level, lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 H.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return lam, np.transpose(H, (0, 2, 1)).copy()


def _op(name):
    fn = getattr(lib(), name)

    def call(prob, *arrays):
        return check(fn(prob, *[ptr(a) for a in arrays]))
    call.__name__ = name
    return call


def sdg_apply_viscous(prob, u, y):
    return _op("sdg_apply_viscous")(prob, u, y)


def sdg_residual_viscous(prob, b, u, r):
    return _op("sdg_residual_viscous")(prob, b, u, r)


def sdg_apply_viscous_f32(prob, u, y):
    return _op("sdg_apply_viscous_f32")(prob, u, y)


def sdg_apply_div(prob, u, q):
    return _op("sdg_apply_div")(prob, u, q)


def sdg_apply_grad(prob, p, v):
    return _op("sdg_apply_grad")(prob, p, v)


def sdg_apply_blockjacobi(prob, r, z):
    return _op("sdg_apply_blockjacobi")(prob, r, z)


def sdg_get_blocks(prob, blocks):
    return _op("sdg_get_blocks")(prob, blocks)


def sdg_get_blocks_noalloc(prob, blocks):
    return _op("sdg_get_blocks_noalloc")(prob, blocks)


def sdg_p_restrict(prob, r, rc):
    return _op("sdg_p_restrict")(prob, r, rc)


def sdg_p_prolong_add(prob, ec, u):
    return _op("sdg_p_prolong_add")(prob, ec, u)


def sdg_get_coarse_stencil(prob, level, st):
    nx, ny = ctypes.c_int(), ctypes.c_int()
    check(lib().sdg_get_coarse_stencil(prob, level, ptr(st), ctypes.byref(nx), ctypes.byref(ny)))
    return nx.value, ny.value


def sdg_vcycle(prob, b, x):
    return _op("sdg_vcycle")(prob, b, x)


def sdg_assemble_rhs(prob, f, g, F, G):
    return check(lib().sdg_assemble_rhs(prob, ptr(f), ptr(g), ptr(F), ptr(G)))


def _stats_out(st, nb):
    d = [st[i].as_dict() for i in range(nb)]
    return d[0] if nb == 1 else d


def sdg_solve_viscous_dev(prob, f, g, u):
    """Returns (rc, stats); stats is a dict, or a list of nbatch dicts."""
    nb = sdg_problem_batch(prob)
    st = (sdg_stats * nb)()
    rc = check(lib().sdg_solve_viscous_dev(prob, ptr(f), ptr(g), ptr(u), st))
    return rc, _stats_out(st, nb)


def sdg_solve_stokes_dev(prob, f, g, u, p):
    nb = sdg_problem_batch(prob)
    st = (sdg_stats * nb)()
    rc = check(lib().sdg_solve_stokes_dev(prob, ptr(f), ptr(g), ptr(u), ptr(p), st))
    return rc, _stats_out(st, nb)


def sdg_solve_viscous_ext_dev(prob, f, g, u_hi, u_lo):
    nb = sdg_problem_batch(prob)
    st = (sdg_stats * nb)()
    rc = check(lib().sdg_solve_viscous_ext_dev(prob, ptr(f), ptr(g), ptr(u_hi), ptr(u_lo), st))
    return rc, _stats_out(st, nb)


def sdg_solve_stokes_ext_dev(prob, f, g, u_hi, u_lo, p_hi, p_lo):
    nb = sdg_problem_batch(prob)
    st = (sdg_stats * nb)()
    rc = check(lib().sdg_solve_stokes_ext_dev(prob, ptr(f), ptr(g), ptr(u_hi), ptr(u_lo), ptr(p_hi),
                                              ptr(p_lo), st))
    return rc, _stats_out(st, nb)


def sdg_residual_ext(prob, stokes, b, x_hi, x_lo, r):
    return check(lib().sdg_residual_ext(prob, int(stokes), ptr(b), ptr(x_hi), ptr(x_lo), ptr(r)))


def sdg_abs_apply(prob, stokes, x, y):
    return check(lib().sdg_abs_apply(prob, int(stokes), ptr(x), ptr(y)))


def sdg_solve_viscous_batch(ctx, meshes, opts, etas, fs, with_lo=False):
    """n solves of (possibly) different meshes and orders; host numpy
    inputs.  Returns (rc, [u_i], [u_lo_i] or None, [stats_i])."""
    n = len(meshes)
    marr = (sdg_mesh * n)(*meshes)
    etas = [np.ascontiguousarray(e, dtype=np.float64) for e in etas]
    fs = [np.ascontiguousarray(f, dtype=np.float64).reshape(-1) for f in fs]
    us = [np.empty(f.size) for f in fs]
    los = [np.empty(f.size) for f in fs] if with_lo else None
    PA = ctypes.c_void_p * n
    st = (sdg_stats * n)()
    rc = check(lib().sdg_solve_viscous_batch(ctx, n, marr, ctypes.byref(opts), PA(*[e.ctypes.data for e in etas]),
                                             PA(*[f.ctypes.data for f in fs]), PA(*[u.ctypes.data for u in us]),
                                             PA(*[l.ctypes.data for l in los]) if with_lo else None, st))
    return rc, us, los, [st[i].as_dict() for i in range(n)]


def sdg_solve_viscous(ctx, mesh, opts, eta, f, g, u):
    st = sdg_stats()
    rc = check(lib().sdg_solve_viscous(ctx, ctypes.byref(mesh), ctypes.byref(opts), ptr(eta), ptr(f),
                                       ptr(g), ptr(u), ctypes.byref(st)))
    return rc, st.as_dict()


def sdg_solve_stokes(ctx, mesh, opts, eta, f, g, u, p):
    st = sdg_stats()
    rc = check(lib().sdg_solve_stokes(ctx, ctypes.byref(mesh), ctypes.byref(opts), ptr(eta), ptr(f),
                                      ptr(g), ptr(u), ptr(p), ctypes.byref(st)))
    return rc, st.as_dict()


def sdg_uniform_pm1(ctx, seed, n, out, stream=None):
    return check(lib().sdg_uniform_pm1(ctx, ctypes.c_uint64(seed), n, ptr(out), stream))


# ---- request server ------------------------------------------------------------
def sdg_server_create(ctx, slots=4, max_batch=16, bypass=8, mem_budget=0, combine=0):
    cfg = sdg_server_config(slots, max_batch, bypass, combine, mem_budget)
    h = ctypes.c_void_p()
    check(lib().sdg_server_create(ctx, ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def sdg_server_destroy(srv):
    lib().sdg_server_destroy(srv)


def _host(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def sdg_submit(srv, mesh, opts, kind, eta, f, g=None):
    """Host numpy inputs (copied by the library); returns a request handle."""
    eta, f, g = _host(eta), _host(f), _host(g)
    h = ctypes.c_void_p()
    check(lib().sdg_submit(srv, ctypes.byref(mesh), ctypes.byref(opts), kind, eta.ctypes.data,
                           f.ctypes.data, None if g is None else g.ctypes.data, ctypes.byref(h)))
    return h.value


def sdg_poll(req):
    d = I()
    check(lib().sdg_poll(req, ctypes.byref(d)))
    return bool(d.value)


def sdg_wait(req, nu, np_=0):
    """-> (rc, u, p, stats dict, info dict); blocks until the request is done."""
    u = np.empty(nu)
    p = np.empty(max(np_, 0)) if np_ else None
    st = sdg_stats()
    info = sdg_req_info()
    rc = check(lib().sdg_wait(req, u.ctypes.data, None if p is None else p.ctypes.data,
                              ctypes.byref(st), ctypes.byref(info)))
    return rc, u, p, st.as_dict(), info.as_dict()


def sdg_req_free(req):
    lib().sdg_req_free(req)


def sdg_server_stats(srv):
    c = ctypes.c_int64()
    pb = ctypes.c_size_t()
    busy = I()
    bud = ctypes.c_size_t()
    check(lib().sdg_server_stats(srv, ctypes.byref(c), ctypes.byref(pb), ctypes.byref(busy), ctypes.byref(bud)))
    return {"completed": c.value, "peak_bytes": pb.value, "peak_busy": busy.value, "budget": bud.value}


def sdg_server_launch_stats(srv):
    n, c, w, g = ctypes.c_int64(), ctypes.c_int64(), I(), ctypes.c_int64()
    check(lib().sdg_server_launch_stats(srv, ctypes.byref(n), ctypes.byref(c), ctypes.byref(w), ctypes.byref(g)))
    return {"launches": n.value, "combined": c.value, "max_width": w.value, "graphs": g.value}


def sdg_admission_simulate(arrival_ms, service_ms, nbytes, slots, budget, bypass):
    a = np.ascontiguousarray(arrival_ms, dtype=np.float64)
    sv = np.ascontiguousarray(service_ms, dtype=np.float64)
    by = np.ascontiguousarray(nbytes, dtype=np.uint64)
    out = np.empty(len(a))
    check(lib().sdg_admission_simulate(len(a), a.ctypes.data, sv.ctypes.data, by.ctypes.data, slots,
                                       int(budget), bypass, out.ctypes.data))
    return out


TILE_APPLY, TILE_RESIDUAL = 0, 1


def sdg_tile_variants(k):
    n = I()
    check(lib().sdg_tile_variants(k, ctypes.byref(n)))
    return n.value


def sdg_tile_shape(k, variant):
    tx, ty = I(), I()
    check(lib().sdg_tile_shape(k, variant, ctypes.byref(tx), ctypes.byref(ty)))
    return tx.value, ty.value


def sdg_get_tile(prob, kernel, precision):
    v = I()
    check(lib().sdg_get_tile(prob, kernel, precision, ctypes.byref(v)))
    return v.value


def sdg_set_tile(prob, kernel, precision, variant):
    return check(lib().sdg_set_tile(prob, kernel, precision, variant))


def sdg_autotune(prob, reps=20):
    """-> ({(kernel, precision): variant}, {(kernel, precision): us}) for
    kernel in (apply, residual) and precision in (FP64, FP32)."""
    v = (I * 4)()
    us = (ctypes.c_double * 4)()
    check(lib().sdg_autotune(prob, reps, v, us))
    keys = [(TILE_APPLY, FP64), (TILE_APPLY, FP32), (TILE_RESIDUAL, FP64), (TILE_RESIDUAL, FP32)]
    return ({k: v[i] for i, k in enumerate(keys) if v[i] >= 0},
            {k: us[i] for i, k in enumerate(keys) if v[i] >= 0})


TRACE_SIP_APPLY, TRACE_SIP_RESIDUAL, TRACE_SMOOTHER, TRACE_COARSE_TAIL = 0, 1, 2, 3
TRACE_NAMES = {TRACE_SIP_APPLY: "sip_apply", TRACE_SIP_RESIDUAL: "sip_residual",
               TRACE_SMOOTHER: "block_jacobi_smoother", TRACE_COARSE_TAIL: "coarse_tail"}


def sdg_trace_enable(ctx, on):
    return check(lib().sdg_trace_enable(ctx, int(on)))


def sdg_trace_read(ctx, kclass):
    """-> (launches, total_ms, bytes) of one traced kernel class."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    by = ctypes.c_double()
    check(lib().sdg_trace_read(ctx, kclass, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
    return n.value, ms.value, by.value


# ---- convenience object ------------------------------------------------------
class Problem:
    """A set-up problem (or batch of problems on one mesh: eta of shape
    [nbatch, nel]) on the current torch stream; device tensors in/out."""

    def __init__(self, ctx, nx, ny, k, eta, bc=(NAVIER,) * 4, lx=1.0, ly=1.0, **options):
        import torch
        self.torch = torch
        self.mesh = make_mesh(nx, ny, k, bc, lx, ly)
        self.opts = make_options(**options)
        self.nx, self.ny, self.k = nx, ny, k
        self.nel = nx * ny
        self.nb = 2 * (k + 1) ** 2
        eta = torch.as_tensor(eta, dtype=torch.float64, device="cuda").contiguous()
        self.nbatch = eta.numel() // self.nel
        assert eta.numel() == self.nbatch * self.nel
        self.nu = self.nel * self.nb * self.nbatch
        self.np = self.nel * k * k * self.nbatch
        self.eta = eta.reshape(-1)
        self.ctx = ctx
        self.h = sdg_problem_create_batch(ctx, self.mesh, self.opts, self.nbatch, self.eta,
                                          current_stream())

    def close(self):
        if self.h:
            sdg_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def zeros(self, n, dtype=None):
        return self.torch.zeros(n, dtype=dtype or self.torch.float64, device="cuda")

    def apply(self, u):
        y = self.zeros(self.nu)
        sdg_apply_viscous(self.h, u, y)
        return y

    def solve_viscous(self, f, g=None):
        u = self.zeros(self.nu)
        rc, st = sdg_solve_viscous_dev(self.h, f, g, u)
        return u, st

    def solve_stokes(self, f, g=None):
        u = self.zeros(self.nu)
        p = self.zeros(max(self.np, 1))
        rc, st = sdg_solve_stokes_dev(self.h, f, g, u, p)
        return u, p[: self.np], st
