"""Python binding of liblagot (argument marshalling only).

Every computation runs in the HIP kernels behind the C-ABI declared in
include/lagot.h; PyTorch only provides device memory and the stream. The
binding raises if the library has not been built: there is no CPU fallback.

  ctx = Context()                                   # lagot_create on the current device/stream
  out = ctx.cells(x, y, z, psi)                     # lagot_cells
  st  = ctx.solve(x, y, z, nu, psi)                 # lagot_solve, psi updated in place
  st  = ctx.newton_step(x, y, z, nu, psi)           # lagot_newton_step
  sts = ctx.solve_batched(offsets, x, y, z, nu, psi, boxes)   # lagot_solve_batched
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblagot.so")
_lib = None

OK, EINVAL, EEMPTY, ENOCONV, ELINESEARCH, ECAPACITY, ESINGULAR, EHIP = 0, -1, -2, -3, -4, -5, -6, -7

EXPORTS = ["lagot_default_opts", "lagot_create", "lagot_destroy", "lagot_cells", "lagot_newton_step", "lagot_solve",
           "lagot_solve_batched", "lagot_solve_moved", "lagot_set_threads_per_cell", "lagot_set_cg_shape", "lagot_set_cg_split", "lagot_last_fallback_cells", "lagot_last_flag_counts", "lagot_last_pass_counts", "lagot_last_kernel_times", "lagot_last_deferred", "lagot_centroids", "lagot_cells_paper_k", "lagot_set_domain", "lagot_set_domain_pieces", "lagot_last_cell_kernel_ms",
           "lagot_p1_laplacian", "lagot_default_fluid_params", "lagot_fluid_velocity", "lagot_fluid_step",
           "lagot_mlp_set_params", "lagot_mlp_get_params", "lagot_features", "lagot_mlp_forward", "lagot_mlp_forward_noalloc",
           "lagot_mlp_train_step", "lagot_mlp_last_grads", "lagot_strerror"]
MLP_NPARAMS = 41473
NOALLOC_MAX_ROWS = 32768  # LAGOT_NOALLOC_MAX_ROWS: rows of lagot_mlp_forward_noalloc's static buffers


class Box(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3)]


class FluidParams(ctypes.Structure):
    """lagot_fluid_params: the velocity update of the fluid step (section 5, eq. (4))."""
    _fields_ = [("dt", ctypes.c_double), ("eps", ctypes.c_double), ("gamma", ctypes.c_double),
                ("mu", ctypes.c_double), ("gravity", ctypes.c_double * 3), ("cg_rtol", ctypes.c_double),
                ("cg_max_iter", ctypes.c_int), ("reserved", ctypes.c_int)]


def default_fluid_params(**kw) -> FluidParams:
    p = FluidParams()
    load().lagot_default_fluid_params(ctypes.byref(p))
    for k, v in kw.items():
        if k == "gravity":
            p.gravity = (ctypes.c_double * 3)(*[float(a) for a in v])
        else:
            setattr(p, k, v)
    return p


class Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_newton", ctypes.c_int), ("max_halvings", ctypes.c_int),
                ("cg_rtol", ctypes.c_double), ("cg_max_iter", ctypes.c_int), ("threads_per_cell", ctypes.c_int),
                ("verbose", ctypes.c_int), ("use_learned", ctypes.c_int), ("empty_start_fallback", ctypes.c_int),
                ("autotune", ctypes.c_int), ("use_graph", ctypes.c_int), ("residual_test", ctypes.c_int),
                ("continuation", ctypes.c_int), ("stage_newton", ctypes.c_int), ("stage_tol", ctypes.c_double),
                ("step_start", ctypes.c_int), ("reserved", ctypes.c_int), ("stage_step", ctypes.c_double),
                ("stage_gtol", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("newton_iters", ctypes.c_int), ("evals", ctypes.c_int),
                ("halvings", ctypes.c_int), ("cg_iters", ctypes.c_int), ("fallback_cells", ctypes.c_int),
                ("failed_cells", ctypes.c_int), ("cell_launches", ctypes.c_int), ("learned_accepted", ctypes.c_int),
                ("default_start", ctypes.c_int), ("repaired_start", ctypes.c_int), ("stages", ctypes.c_int),
                ("max_rel_err", ctypes.c_double), ("grad_norm", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("ms_eval", ctypes.c_double), ("ms_linear", ctypes.c_double),
                ("ms_cell_kernel", ctypes.c_double), ("ms_learned", ctypes.c_double),
                ("reserved_d", ctypes.c_double * 1)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if not k.startswith("reserved")}


class LagotError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


def load():
    """Load liblagot.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2601_05765_amd.build.build()")
        lib = ctypes.CDLL(LIB_PATH)
        P, I64, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        lib.lagot_default_opts.argtypes = [ctypes.POINTER(Opts)]
        lib.lagot_default_opts.restype = None
        lib.lagot_create.argtypes = [ctypes.POINTER(P), I, P]
        lib.lagot_create.restype = I
        lib.lagot_destroy.argtypes = [P]
        lib.lagot_destroy.restype = None
        lib.lagot_cells.argtypes = [P, I64, P, P, P, P, Box, P, P, P, P, P, P, I64, ctypes.POINTER(I64)]
        lib.lagot_cells.restype = I
        for name in ("lagot_newton_step", "lagot_solve"):
            f = getattr(lib, name)
            f.argtypes = [P, I64, P, P, P, P, Box, P, ctypes.POINTER(Opts), ctypes.POINTER(Stats)]
            f.restype = I
        lib.lagot_solve_batched.argtypes = [P, ctypes.c_int32, ctypes.POINTER(I64), P, P, P, P, ctypes.POINTER(Box),
                                            P, ctypes.POINTER(Opts), ctypes.POINTER(Stats)]
        lib.lagot_solve_moved.argtypes = [P, I64, P, P, P, P, P, P, P, Box, P, ctypes.POINTER(Opts),
                                          ctypes.POINTER(Stats)]
        lib.lagot_solve_moved.restype = I
        lib.lagot_solve_batched.restype = I
        lib.lagot_mlp_set_params.argtypes = [P, P]
        lib.lagot_mlp_get_params.argtypes = [P, P]
        lib.lagot_mlp_last_grads.argtypes = [P, P]
        lib.lagot_features.argtypes = [P, I64, P, P, P, P, P, Box, P, P]
        lib.lagot_mlp_forward.argtypes = [P, I64, P, P]
        lib.lagot_mlp_forward_noalloc.argtypes = [P, I64, P, P]
        lib.lagot_mlp_train_step.argtypes = [P, I64, P, P, P, ctypes.c_int32, ctypes.c_float,
                                             ctypes.POINTER(ctypes.c_float)]
        for f in ("lagot_mlp_set_params", "lagot_mlp_get_params", "lagot_mlp_last_grads", "lagot_features",
                  "lagot_mlp_forward", "lagot_mlp_forward_noalloc", "lagot_mlp_train_step"):
            getattr(lib, f).restype = I
        lib.lagot_set_threads_per_cell.argtypes = [P, I]
        lib.lagot_set_threads_per_cell.restype = I
        lib.lagot_set_cg_shape.argtypes = [P, I, I]
        lib.lagot_set_cg_shape.restype = I
        lib.lagot_set_cg_split.argtypes = [P, I]
        lib.lagot_set_cg_split.restype = I
        lib.lagot_set_domain.argtypes = [P, ctypes.c_int, P]
        lib.lagot_set_domain.restype = I
        lib.lagot_set_domain_pieces.argtypes = [P, ctypes.c_int, P, P, P, ctypes.c_int]
        lib.lagot_set_domain_pieces.restype = I
        lib.lagot_centroids.argtypes = [P, I64, P, P, P, P, Box, P, P]
        lib.lagot_centroids.restype = I
        lib.lagot_cells_paper_k.argtypes = [P, I64, P, P, P, P, Box, P, P]
        lib.lagot_cells_paper_k.restype = I
        lib.lagot_p1_laplacian.argtypes = [P, I64, P, P, P, P, Box, P, ctypes.c_double, P, P]
        lib.lagot_p1_laplacian.restype = I
        lib.lagot_default_fluid_params.argtypes = [ctypes.POINTER(FluidParams)]
        lib.lagot_default_fluid_params.restype = None
        lib.lagot_fluid_velocity.argtypes = [P, I64, P, P, P, P, Box, P, P, P, ctypes.POINTER(FluidParams), P, P,
                                             ctypes.POINTER(ctypes.c_int32 * 3)]
        lib.lagot_fluid_velocity.restype = I
        lib.lagot_fluid_step.argtypes = [P, I64, P, P, P, P, Box, P, P, P, P, ctypes.POINTER(FluidParams),
                                         ctypes.POINTER(Opts), ctypes.POINTER(Stats), ctypes.POINTER(ctypes.c_int32 * 3)]
        lib.lagot_fluid_step.restype = I
        lib.lagot_last_flag_counts.argtypes = [P, P]
        lib.lagot_last_flag_counts.restype = I
        lib.lagot_last_pass_counts.argtypes = [P, P]
        lib.lagot_last_pass_counts.restype = I
        lib.lagot_last_kernel_times.argtypes = [P, P]
        lib.lagot_last_kernel_times.restype = I
        lib.lagot_last_deferred.argtypes = [P, P, I64, ctypes.POINTER(I64)]
        lib.lagot_last_deferred.restype = I
        lib.lagot_last_fallback_cells.argtypes = [P]
        lib.lagot_last_fallback_cells.restype = I
        lib.lagot_last_cell_kernel_ms.argtypes = [P]
        lib.lagot_last_cell_kernel_ms.restype = ctypes.c_double
        lib.lagot_strerror.argtypes = [I]
        lib.lagot_strerror.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def strerror(code: int) -> str:
    return load().lagot_strerror(int(code)).decode()


def default_opts(**kw) -> Opts:
    o = Opts()
    load().lagot_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def make_box(box=((0.0, 0.0, 0.0), (1.0, 1.0, 1.0))) -> Box:
    b = Box()
    for a in range(3):
        b.lo[a] = float(box[0][a])
        b.hi[a] = float(box[1][a])
    return b


def _dev(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """A lagot context bound to one device and one stream (default: torch's current)."""

    def __init__(self, device: int | None = None, stream=None):
        import torch
        lib = load()
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        rc = lib.lagot_create(ctypes.byref(h), self.device, ctypes.c_void_p(stream.cuda_stream))
        if rc != OK:
            raise LagotError(rc, "lagot_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().lagot_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def cells(self, x, y, z, psi, box=((0, 0, 0), (1, 1, 1)), csr: bool = True, walls: bool = True,
              sph: bool = True, nnz_per_cell: int = 24):
        """lagot_cells: volumes, spherical areas, wall areas and the facet CSR (caller order)."""
        import torch
        n = x.shape[0]
        dev = x.device
        args = [_dev(x, torch.float32, "x"), _dev(y, torch.float32, "y"), _dev(z, torch.float32, "z"),
                _dev(psi, torch.float64, "psi")]
        vol = torch.empty(n, dtype=torch.float64, device=dev)
        K = torch.empty(n, dtype=torch.float64, device=dev) if sph else None
        nwall = getattr(self, "_nwall", 6)
        W = torch.empty(n * nwall, dtype=torch.float32, device=dev) if walls else None
        out = {"vol": vol}
        lib = load()
        cap = nnz_per_cell * n
        while True:
            nnz = ctypes.c_int64(0)
            if csr:
                rp = torch.empty(n + 1, dtype=torch.int64, device=dev)
                col = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
                fa = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
                ptrs = [ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(col.data_ptr()),
                        ctypes.c_void_p(fa.data_ptr())]
            else:
                ptrs = [None, None, None]
            rc = lib.lagot_cells(self._h, n, *args, make_box(box), ctypes.c_void_p(vol.data_ptr()),
                                 ctypes.c_void_p(K.data_ptr()) if K is not None else None,
                                 ctypes.c_void_p(W.data_ptr()) if W is not None else None, *ptrs, cap,
                                 ctypes.byref(nnz))
            if rc == ECAPACITY and csr and nnz.value > cap:
                cap = int(nnz.value)
                continue
            if rc != OK:
                raise LagotError(rc, "lagot_cells")
            break
        if K is not None:
            out["sph"] = K
        if W is not None:
            out["walls"] = W.view(n, nwall)
        if csr:
            out["row_ptr"], out["col"], out["area"] = rp, col[: nnz.value], fa[: nnz.value]
        out["nnz"] = int(nnz.value)
        return out

    def centroids(self, x, y, z, psi, box=((0, 0, 0), (1, 1, 1))):
        """lagot_centroids: (volumes [n], centroids [n, 3]) in caller order, float64."""
        import torch
        n = x.shape[0]
        args = [_dev(x, torch.float32, "x"), _dev(y, torch.float32, "y"), _dev(z, torch.float32, "z"),
                _dev(psi, torch.float64, "psi")]
        vol = torch.empty(n, dtype=torch.float64, device=x.device)
        cen = torch.empty((n, 3), dtype=torch.float64, device=x.device)
        rc = load().lagot_centroids(self._h, n, *args, make_box(box), ctypes.c_void_p(vol.data_ptr()),
                                    ctypes.c_void_p(cen.data_ptr()))
        if rc != OK:
            raise LagotError(rc, "lagot_centroids")
        return vol, cen

    def cells_paper_k(self, x, y, z, psi, box=((0, 0, 0), (1, 1, 1))):
        """lagot_cells_paper_k: (volumes [n], spherical areas [n]) in caller order, float64,
        with |K| by section 3.3's own route (interior point, projected facets, Gauss-Bonnet)."""
        import torch
        n = x.shape[0]
        args = [_dev(x, torch.float32, "x"), _dev(y, torch.float32, "y"), _dev(z, torch.float32, "z"),
                _dev(psi, torch.float64, "psi")]
        vol = torch.empty(n, dtype=torch.float64, device=x.device)
        sph = torch.empty(n, dtype=torch.float64, device=x.device)
        rc = load().lagot_cells_paper_k(self._h, n, *args, make_box(box), ctypes.c_void_p(vol.data_ptr()),
                                        ctypes.c_void_p(sph.data_ptr()))
        if rc != OK:
            raise LagotError(rc, "lagot_cells_paper_k")
        return vol, sph

    def p1_laplacian(self, x, y, z, psi, u, mu=None, mu0: float = 1.0, box=((0, 0, 0), (1, 1, 1))):
        """lagot_p1_laplacian: Lap_mu u ([n, 3] float64, caller order) over the restricted
        Laguerre facets (eq. (3)); mu: per-site coefficients [n] or None (mu0)."""
        import torch
        n = x.shape[0]
        args = [_dev(x, torch.float32, "x"), _dev(y, torch.float32, "y"), _dev(z, torch.float32, "z"),
                _dev(psi, torch.float64, "psi")]
        if tuple(u.shape) != (n, 3) or (mu is not None and tuple(mu.shape) != (n,)):
            raise ValueError("u must be [n, 3] and mu [n]")
        u_p = _dev(u, torch.float64, "u")
        mu_p = None if mu is None else _dev(mu, torch.float64, "mu")
        out = torch.empty((n, 3), dtype=torch.float64, device=x.device)
        rc = load().lagot_p1_laplacian(self._h, n, *args, make_box(box), mu_p, float(mu0), u_p,
                                       ctypes.c_void_p(out.data_ptr()))
        if rc != OK:
            raise LagotError(rc, "lagot_p1_laplacian")
        return out

    def fluid_velocity(self, x, y, z, psi, mass, v, params=None, mu=None, box=((0, 0, 0), (1, 1, 1))):
        """lagot_fluid_velocity: (v_new [n, 3], centroids [n, 3], PCG iterations per
        coordinate) of the semi-implicit velocity update (section 5, eq. (4))."""
        import torch
        n = x.shape[0]
        args = [_dev(x, torch.float32, "x"), _dev(y, torch.float32, "y"), _dev(z, torch.float32, "z"),
                _dev(psi, torch.float64, "psi")]
        if tuple(v.shape) != (n, 3) or tuple(mass.shape) != (n,) or (mu is not None and tuple(mu.shape) != (n,)):
            raise ValueError("mass and mu must be [n], v [n, 3]")
        m_p = _dev(mass, torch.float64, "mass")
        v_p = _dev(v, torch.float64, "v")
        mu_p = None if mu is None else _dev(mu, torch.float64, "mu")
        prm = params if params is not None else default_fluid_params()
        out = torch.empty((n, 3), dtype=torch.float64, device=x.device)
        cen = torch.empty((n, 3), dtype=torch.float64, device=x.device)
        it = (ctypes.c_int32 * 3)()
        rc = load().lagot_fluid_velocity(self._h, n, *args, make_box(box), m_p, mu_p, v_p, ctypes.byref(prm),
                                         ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(cen.data_ptr()),
                                         ctypes.byref(it))
        if rc != OK:
            raise LagotError(rc, "lagot_fluid_velocity")
        return out, cen, list(it)

    def fluid_step(self, x, y, z, nu, psi, mass, v, params=None, opts=None, mu=None, box=((0, 0, 0), (1, 1, 1))):
        """lagot_fluid_step, in place on x, y, z, psi and v: move the sites with v, re-solve
        the weights, update v (section 5). Returns (stats, PCG iterations per coordinate)."""
        import torch
        n = x.shape[0]
        if tuple(v.shape) != (n, 3) or tuple(mass.shape) != (n,) or (mu is not None and tuple(mu.shape) != (n,)):
            raise ValueError("mass and mu must be [n], v [n, 3]")
        args = [_dev(x, torch.float32, "x"), _dev(y, torch.float32, "y"), _dev(z, torch.float32, "z"),
                _dev(nu, torch.float64, "nu")]
        psi_p = _dev(psi, torch.float64, "psi")
        m_p = _dev(mass, torch.float64, "mass")
        mu_p = None if mu is None else _dev(mu, torch.float64, "mu")
        v_p = _dev(v, torch.float64, "v")
        prm = params if params is not None else default_fluid_params()
        o = opts if opts is not None else default_opts()
        st = Stats()
        it = (ctypes.c_int32 * 3)()
        rc = load().lagot_fluid_step(self._h, n, *args, make_box(box), psi_p, m_p, mu_p, v_p, ctypes.byref(prm),
                                     ctypes.byref(o), ctypes.byref(st), ctypes.byref(it))
        if rc != OK:
            raise LagotError(rc, "lagot_fluid_step")
        return st, list(it)

    def set_domain(self, planes=None) -> None:
        """lagot_set_domain: planes [P, 4] (unit outward normal, c) of the convex domain
        n.x <= c, or None for the box."""
        import numpy as np
        if planes is None:
            arr, p = None, 0
        else:
            arr = np.ascontiguousarray(planes, np.float64).reshape(-1, 4)
            p = arr.shape[0]
        rc = load().lagot_set_domain(self._h, p, arr.ctypes.data_as(ctypes.c_void_p) if p else None)
        if rc != OK:
            raise LagotError(rc, "lagot_set_domain")
        self._nwall = max(p, 0) if p else 6

    def set_domain_pieces(self, pieces, nwalls: int) -> None:
        """lagot_set_domain_pieces: a non-convex domain as the union of convex pieces.
        ``pieces`` is a list of (planes [P_k, 4] (unit outward normal, c), wall_id [P_k]
        (wall index, or -1 for a plane between pieces)); ``nwalls`` walls in all."""
        import numpy as np
        planes = np.ascontiguousarray(np.concatenate([np.asarray(p, np.float64).reshape(-1, 4) for p, _ in pieces]))
        wid = np.ascontiguousarray(np.concatenate([np.asarray(w, np.int32).reshape(-1) for _, w in pieces]), np.int32)
        off = np.ascontiguousarray(np.cumsum([0] + [np.asarray(p).reshape(-1, 4).shape[0] for p, _ in pieces]),
                                   np.int32)
        rc = load().lagot_set_domain_pieces(self._h, len(pieces), off.ctypes.data_as(ctypes.c_void_p),
                                            planes.ctypes.data_as(ctypes.c_void_p),
                                            wid.ctypes.data_as(ctypes.c_void_p), int(nwalls))
        if rc != OK:
            raise LagotError(rc, "lagot_set_domain_pieces")
        self._nwall = int(nwalls)

    def set_cg_shape(self, lanes_per_row: int, rows_per_block: int) -> None:
        rc = load().lagot_set_cg_shape(self._h, int(lanes_per_row), int(rows_per_block))
        if rc != OK:
            raise LagotError(rc, "lagot_set_cg_shape")

    def set_cg_split(self, mode: int) -> None:
        """lagot_set_cg_split: 0 auto (two launches per PCG iteration for large instances),
        1 always one launch, 2 always two."""
        rc = load().lagot_set_cg_split(self._h, int(mode))
        if rc != OK:
            raise LagotError(rc, "lagot_set_cg_split")

    def set_threads_per_cell(self, tpc: int) -> None:
        rc = load().lagot_set_threads_per_cell(self._h, int(tpc))
        if rc != OK:
            raise LagotError(rc, "lagot_set_threads_per_cell")

    # ---- learned warm start ----
    def mlp_set_params(self, params):
        import torch
        rc = load().lagot_mlp_set_params(self._h, _dev(params, torch.float32, "params"))
        if rc != OK:
            raise LagotError(rc, "lagot_mlp_set_params")

    def mlp_get_params(self):
        import torch
        out = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=f"cuda:{self.device}")
        rc = load().lagot_mlp_get_params(self._h, ctypes.c_void_p(out.data_ptr()))
        if rc != OK:
            raise LagotError(rc, "lagot_mlp_get_params")
        return out

    def mlp_last_grads(self):
        import torch
        out = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=f"cuda:{self.device}")
        rc = load().lagot_mlp_last_grads(self._h, ctypes.c_void_p(out.data_ptr()))
        if rc != OK:
            raise LagotError(rc, "lagot_mlp_last_grads")
        return out

    def features(self, x, y, z, psi_prev, nu, box=((0, 0, 0), (1, 1, 1)), want_nbr: bool = True):
        """lagot_features: (nbr int32 [n,16] caller indices, inputs bf16-as-int16 [n,64])."""
        import torch
        n = x.shape[0]
        nbr = torch.empty((n, 16), dtype=torch.int32, device=x.device) if want_nbr else None
        feats = torch.empty((n, 64), dtype=torch.int16, device=x.device)
        rc = load().lagot_features(self._h, n, _dev(x, torch.float32, "x"), _dev(y, torch.float32, "y"),
                                   _dev(z, torch.float32, "z"), _dev(psi_prev, torch.float64, "psi_prev"),
                                   _dev(nu, torch.float64, "nu"), make_box(box),
                                   ctypes.c_void_p(nbr.data_ptr()) if nbr is not None else None,
                                   ctypes.c_void_p(feats.data_ptr()))
        if rc != OK:
            raise LagotError(rc, "lagot_features")
        return nbr, feats

    def mlp_forward(self, feats):
        import torch
        out = torch.empty(feats.shape[0], dtype=torch.float32, device=feats.device)
        rc = load().lagot_mlp_forward(self._h, feats.shape[0], _dev(feats, torch.int16, "feats"),
                                      ctypes.c_void_p(out.data_ptr()))
        if rc != OK:
            raise LagotError(rc, "lagot_mlp_forward")
        return out

    def mlp_forward_noalloc(self, feats, out):
        """lagot_mlp_forward_noalloc: the network output of the rows of feats into the
        caller's out (float32 [m], device); enqueued on the context's stream, not
        synchronised."""
        import torch
        if out.dtype != torch.float32 or not out.is_contiguous() or out.shape[0] < feats.shape[0]:
            raise ValueError("out: contiguous float32 with at least one value per row")
        rc = load().lagot_mlp_forward_noalloc(self._h, feats.shape[0], _dev(feats, torch.int16, "feats"),
                                              ctypes.c_void_p(out.data_ptr()))
        if rc != OK:
            raise LagotError(rc, "lagot_mlp_forward_noalloc")
        return out

    def mlp_train_step(self, feats, targets, batch_idx, lr: float, want_loss: bool = True):
        import torch
        loss = ctypes.c_float(0.0)
        rc = load().lagot_mlp_train_step(self._h, feats.shape[0], _dev(feats, torch.int16, "feats"),
                                         _dev(targets, torch.float32, "targets"),
                                         _dev(batch_idx, torch.int32, "batch_idx"), batch_idx.shape[0],
                                         float(lr), ctypes.byref(loss) if want_loss else None)
        if rc != OK:
            raise LagotError(rc, "lagot_mlp_train_step")
        return float(loss.value) if want_loss else None

    def last_fallback_cells(self) -> int:
        return int(load().lagot_last_fallback_cells(self._h))

    FLAG_NAMES = ("empty", "candidates", "planes", "vertices", "topology", "walk", "facets", "precision")

    def last_flag_counts(self) -> dict:
        """lagot_last_flag_counts: {"final": {name: cells}, "float64_reasons": {name: cells}}."""
        buf = (ctypes.c_int64 * 16)()
        rc = load().lagot_last_flag_counts(self._h, ctypes.cast(buf, ctypes.c_void_p))
        if rc != OK:
            raise LagotError(rc, "lagot_last_flag_counts")
        return {"final": {k: int(buf[i]) for i, k in enumerate(self.FLAG_NAMES)},
                "float64_reasons": {k: int(buf[8 + i]) for i, k in enumerate(self.FLAG_NAMES)}}

    def last_pass_counts(self) -> dict:
        """lagot_last_pass_counts: cells of the last evaluation deferred as crowded, cells
        listed for the float64 pass, and whether the crowded pass ran."""
        buf = (ctypes.c_int64 * 3)()
        rc = load().lagot_last_pass_counts(self._h, ctypes.cast(buf, ctypes.c_void_p))
        if rc != OK:
            raise LagotError(rc, "lagot_last_pass_counts")
        return {"crowded": int(buf[0]), "float64": int(buf[1]), "crowded_pass": bool(buf[2])}

    def last_kernel_times(self) -> dict:
        """lagot_last_kernel_times: summed ms and launches of the float32 cell kernel and of the
        crowded-cell pass in the last call."""
        buf = (ctypes.c_double * 5)()
        rc = load().lagot_last_kernel_times(self._h, ctypes.cast(buf, ctypes.c_void_p))
        if rc != OK:
            raise LagotError(rc, "lagot_last_kernel_times")
        return {"fast_ms": buf[0], "fast_launches": int(buf[1]), "crowd_ms": buf[2], "crowd_launches": int(buf[3]),
                "crowd_cells": int(buf[4])}

    def last_deferred(self, cap: int = 1 << 30):
        """lagot_last_deferred: caller indices (numpy int32) of the cells the last evaluation
        deferred as crowded."""
        import numpy as np
        cnt = ctypes.c_int64(0)
        rc = load().lagot_last_deferred(self._h, None, 0, ctypes.byref(cnt))
        if rc != OK:
            raise LagotError(rc, "lagot_last_deferred")
        k = int(min(cnt.value, cap))
        out = np.zeros(k, dtype=np.int32)
        if k:
            rc = load().lagot_last_deferred(self._h, out.ctypes.data_as(ctypes.c_void_p), k, ctypes.byref(cnt))
            if rc != OK:
                raise LagotError(rc, "lagot_last_deferred")
        return out

    def last_cell_kernel_ms(self) -> float:
        return float(load().lagot_last_cell_kernel_ms(self._h))

    def _newton(self, fn, x, y, z, nu, psi, box, opts, check):
        import torch
        args = [_dev(x, torch.float32, "x"), _dev(y, torch.float32, "y"), _dev(z, torch.float32, "z"),
                _dev(nu, torch.float64, "nu")]
        st = Stats()
        o = opts if opts is not None else default_opts()
        rc = fn(self._h, x.shape[0], *args, make_box(box), _dev(psi, torch.float64, "psi"), ctypes.byref(o),
                ctypes.byref(st))
        if check and rc != OK:
            raise LagotError(rc, fn.__name__)
        return st

    def solve(self, x, y, z, nu, psi, box=((0, 0, 0), (1, 1, 1)), opts: Opts | None = None, check: bool = True):
        """lagot_solve: damped Newton to opts.tol; psi (float64, device) is updated in place."""
        return self._newton(load().lagot_solve, x, y, z, nu, psi, box, opts, check)

    def newton_step(self, x, y, z, nu, psi, box=((0, 0, 0), (1, 1, 1)), opts: Opts | None = None,
                    check: bool = True):
        """lagot_newton_step: one damped Newton iteration; psi updated in place."""
        return self._newton(load().lagot_newton_step, x, y, z, nu, psi, box, opts, check)

    def solve_moved(self, x0, y0, z0, x1, y1, z1, nu, psi, box=((0, 0, 0), (1, 1, 1)), opts: Opts | None = None,
                    check: bool = True):
        """lagot_solve_moved: psi (the solution at p0) becomes the solution at p1, in place."""
        import torch
        f32 = [_dev(a, torch.float32, nm) for a, nm in ((x0, "x0"), (y0, "y0"), (z0, "z0"), (x1, "x1"), (y1, "y1"),
                                                         (z1, "z1"))]
        st = Stats()
        o = opts if opts is not None else default_opts()
        rc = load().lagot_solve_moved(self._h, x1.shape[0], *f32, _dev(nu, torch.float64, "nu"), make_box(box),
                                      _dev(psi, torch.float64, "psi"), ctypes.byref(o), ctypes.byref(st))
        if check and rc != OK:
            raise LagotError(rc, "lagot_solve_moved")
        return st

    def solve_batched(self, offsets, x, y, z, nu, psi, boxes=None, opts: Opts | None = None, check: bool = True):
        """lagot_solve_batched: instance b owns rows offsets[b]:offsets[b+1] of the concatenated
        device arrays; psi is updated in place. Returns the per-instance Stats list."""
        import torch
        offs = [int(v) for v in offsets]
        B = len(offs) - 1
        if B < 1:
            raise ValueError("offsets needs at least two entries")
        if boxes is None:
            boxes = [((0, 0, 0), (1, 1, 1))] * B
        if len(boxes) != B:
            raise ValueError("one box per instance")
        c_off = (ctypes.c_int64 * (B + 1))(*offs)
        c_box = (Box * B)(*[make_box(b) for b in boxes])
        stats = (Stats * B)()
        o = opts if opts is not None else default_opts()
        args = [_dev(x, torch.float32, "x"), _dev(y, torch.float32, "y"), _dev(z, torch.float32, "z"),
                _dev(nu, torch.float64, "nu")]
        rc = load().lagot_solve_batched(self._h, B, c_off, *args, c_box, _dev(psi, torch.float64, "psi"),
                                        ctypes.byref(o), stats)
        if check and rc != OK:
            raise LagotError(rc, "lagot_solve_batched")
        return list(stats)
