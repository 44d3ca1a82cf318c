"""ctypes binding of libosm (include/osm.h).

Argument marshalling only: every step of the solver runs in the HIP kernels
of libosm.so.  Device buffers are torch tensors on the handle's device; the
handle is bound to torch's current HIP stream at setup.  There is no CPU
fallback: importing this module raises if libosm.so has not been built.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libosm.so")

OSM_OK, OSM_EINVAL, OSM_ENOMEM, OSM_EHIP = 0, -1, -2, -3
OSM_ENOCONV, OSM_ENONFINITE, OSM_ESTATE, OSM_EUNSUPPORTED = -4, -5, -6, -7
STATUS_NAMES = {0: "OSM_OK", -1: "OSM_EINVAL", -2: "OSM_ENOMEM", -3: "OSM_EHIP",
                -4: "OSM_ENOCONV", -5: "OSM_ENONFINITE", -6: "OSM_ESTATE",
                -7: "OSM_EUNSUPPORTED"}
OSM_TC_ROBIN, OSM_TC_PADE = 0, 1
OSM_CLASSICAL, OSM_PRECOND, OSM_INTERFACE_KRYLOV = 0, 1, 2
OSM_FP64, OSM_C32_REFINE = 0, 1
OSM_IFACE_R, OSM_IFACE_I_MINUS_R, OSM_IFACE_LH, OSM_IFACE_PINV = 0, 1, 2, 3


class osm_problem(ctypes.Structure):
    _fields_ = [("xl", ctypes.c_double), ("xr", ctypes.c_double),
                ("yb", ctypes.c_double), ("yu", ctypes.c_double),
                ("ncx", ctypes.c_int32), ("ncy", ctypes.c_int32),
                ("nsub", ctypes.c_int32),
                ("strip_cells", ctypes.POINTER(ctypes.c_int32)),
                ("lap_coef", ctypes.c_double), ("beta", ctypes.c_double),
                ("tc", ctypes.c_int32), ("p", ctypes.c_double),
                ("p_bc", ctypes.c_double), ("dt", ctypes.c_double),
                ("omega", ctypes.c_double), ("vxx", ctypes.c_double),
                ("vyy", ctypes.c_double), ("pade_m", ctypes.c_int32),
                ("pade_theta", ctypes.c_double)]


class osm_options(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("tol_k", ctypes.c_double), ("tol_k_relative", ctypes.c_int32),
                ("max_k", ctypes.c_int32), ("tol_q", ctypes.c_double),
                ("max_q", ctypes.c_int32), ("fixed_k", ctypes.c_int32),
                ("fixed_q", ctypes.c_int32), ("warm_start", ctypes.c_int32),
                ("tol_gmres", ctypes.c_double), ("gmres_restart", ctypes.c_int32),
                ("max_gmres", ctypes.c_int32), ("guess", ctypes.c_int32),
                ("team", ctypes.c_int32), ("mem_cap", ctypes.c_uint64),
                ("eta_q", ctypes.c_double), ("solve_shape", ctypes.c_int32),
                ("q_estimate", ctypes.c_int32), ("g1_init", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("krylov", ctypes.c_int32),
                ("strip_order", ctypes.c_int32), ("lh_form", ctypes.c_int32)]


class osm_step_stats(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("q_total", ctypes.c_int32),
                ("gmres_total", ctypes.c_int32), ("refine_total", ctypes.c_int32),
                ("fallback_used", ctypes.c_int32), ("last_increment", ctypes.c_double),
                ("mass_before", ctypes.c_double), ("mass_after", ctypes.c_double),
                ("guess_ratio", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class osm_footprint(ctypes.Structure):
    _fields_ = [("device_bytes", ctypes.c_uint64), ("host_bytes", ctypes.c_uint64)]


EXPORTS = ["osm_query", "osm_setup", "osm_factor", "osm_factor_rotating", "osm_step",
           "osm_interface_apply", "osm_set_interface_guess", "osm_get_interface",
           "osm_strip_solve", "osm_get_strip_solution", "osm_get_lh_blocks", "osm_get_factor",
           "osm_get_yfactor", "osm_strip_order", "osm_lh_form",
           "osm_kernel_timing", "osm_kernel_work", "osm_solve_team", "osm_solve_shape",
           "osm_net_nparams", "osm_net_create", "osm_net_set_params", "osm_net_get_params",
           "osm_net_forward", "osm_net_loss_grad", "osm_net_loss_grad_noalloc",
           "osm_net_train_step", "osm_net_destroy",
           "osm_net_last_error", "osm_guess_features", "osm_set_guess_net",
           "osm_factor_timing", "osm_query_batch", "osm_setup_batch", "osm_factor_batch", "osm_step_batch",
           "osm_batch_tuning", "osm_destroy", "osm_last_error"]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    H = ctypes.c_void_p
    P = ctypes.c_void_p
    st = ctypes.c_int
    sig = {
        "osm_query": ([ctypes.POINTER(osm_problem), ctypes.POINTER(osm_options),
                       ctypes.POINTER(osm_footprint)], st),
        "osm_setup": ([ctypes.POINTER(osm_problem), ctypes.POINTER(osm_options), P,
                       ctypes.POINTER(H)], st),
        "osm_factor": ([H, P], st),
        "osm_factor_rotating": ([H, ctypes.c_int32], st),
        "osm_step": ([H, P, ctypes.POINTER(osm_step_stats)], st),
        "osm_interface_apply": ([H, ctypes.c_int, P, P, P], st),
        "osm_set_interface_guess": ([H, P], st),
        "osm_get_interface": ([H, P], st),
        "osm_strip_solve": ([H, P, P], st),
        "osm_get_strip_solution": ([H, P], st),
        "osm_get_lh_blocks": ([H, P], st),
        "osm_get_factor": ([H, P], st),
        "osm_get_yfactor": ([H, P], st),
        "osm_strip_order": ([H], ctypes.c_int32),
        "osm_lh_form": ([H], ctypes.c_int32),
        "osm_solve_team": ([H], ctypes.c_int32),
        "osm_solve_shape": ([H], ctypes.c_int32),
        "osm_kernel_timing": ([H, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_int64)], st),
        "osm_kernel_work": ([H, ctypes.POINTER(ctypes.c_double)], st),
        "osm_factor_timing": ([H, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                               ctypes.POINTER(ctypes.c_double)], st),
        "osm_net_nparams": ([], ctypes.c_int32),
        "osm_net_create": ([ctypes.c_int32, P, ctypes.POINTER(H)], st),
        "osm_net_set_params": ([H, P], st),
        "osm_net_get_params": ([H, ctypes.c_int32, P], st),
        "osm_net_forward": ([H, P, ctypes.c_int32, ctypes.c_int32, P], st),
        "osm_net_loss_grad": ([H, P, P, ctypes.c_int32, ctypes.c_int32, P,
                               ctypes.POINTER(ctypes.c_double)], st),
        "osm_net_loss_grad_noalloc": ([H, P, P, ctypes.c_int32, ctypes.c_int32, P, P], st),
        "osm_net_train_step": ([H, P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                ctypes.POINTER(ctypes.c_double)], st),
        "osm_net_destroy": ([H], None),
        "osm_net_last_error": ([H], ctypes.c_char_p),
        "osm_guess_features": ([H, P, P, P, P, P], st),
        "osm_set_guess_net": ([H, H], st),
        "osm_query_batch": ([ctypes.POINTER(osm_problem), ctypes.c_int32,
                             ctypes.POINTER(osm_options), ctypes.POINTER(osm_footprint)], st),
        "osm_setup_batch": ([ctypes.POINTER(osm_problem), ctypes.c_int32,
                             ctypes.POINTER(osm_options), P, ctypes.POINTER(H)], st),
        "osm_factor_batch": ([H, ctypes.POINTER(ctypes.c_void_p)], st),
        "osm_step_batch": ([H, ctypes.POINTER(ctypes.c_void_p),
                            ctypes.POINTER(osm_step_stats)], st),
        "osm_batch_tuning": ([H, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)], st),
        "osm_destroy": ([H], None),
        "osm_last_error": ([H], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = load_library()


class OsmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(status, handle=None):
    if status != OSM_OK:
        msg = _lib.osm_last_error(handle)
        raise OsmError(status, msg.decode() if msg else "")


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def make_problem(pb):
    """osm_problem from any object with the problem-statement attributes
    (xl, xr, yb, yu, ncx, ncy, nsub, strip_cells, lap_coef, beta, p, p_bc,
    dt and optionally omega, vxx, vyy, tc ("robin" | "pade"), pade_m,
    pade_theta).  Returns (struct, keep-alive)."""
    cells = (ctypes.c_int32 * pb.nsub)(*[int(c) for c in pb.strip_cells])
    tc = {"robin": OSM_TC_ROBIN, "pade": OSM_TC_PADE}[getattr(pb, "tc", "robin")]
    s = osm_problem(pb.xl, pb.xr, pb.yb, pb.yu, pb.ncx, pb.ncy, pb.nsub, cells,
                    pb.lap_coef, pb.beta, tc, pb.p, pb.p_bc, pb.dt,
                    getattr(pb, "omega", 0.0), getattr(pb, "vxx", 0.0),
                    getattr(pb, "vyy", 0.0), int(getattr(pb, "pade_m", 0)),
                    float(getattr(pb, "pade_theta", 0.7853981633974483)))
    return s, cells


def make_options(algo="classical", prec="fp64", tol_k=1e-10, tol_k_relative=False,
                 max_k=2000, tol_q=1e-13, max_q=100, fixed_k=0, fixed_q=0,
                 warm_start=True, tol_gmres=1e-12, gmres_restart=50, max_gmres=1000,
                 guess=0, team=0, mem_cap=0, eta_q=0.0, solve_shape=0, q_estimate=0,
                 g1_init=0, seed=0, krylov="gmres", strip_order="node", lh_form="auto"):
    return osm_options({"classical": OSM_CLASSICAL, "precond": OSM_PRECOND,
                        "interface": OSM_INTERFACE_KRYLOV}[algo],
                       {"fp64": OSM_FP64, "c32": OSM_C32_REFINE}[prec],
                       tol_k, int(tol_k_relative), max_k, tol_q, max_q, fixed_k, fixed_q,
                       int(warm_start), tol_gmres, gmres_restart, max_gmres, guess, team,
                       mem_cap, eta_q, solve_shape, int(q_estimate), int(g1_init),
                       int(seed) & 0xFFFFFFFFFFFFFFFF, {"gmres": 0, "bicgstab": 1}[krylov],
                       {"node": 0, "y": 1, "tuned": 2}[strip_order],
                       {"auto": 0, "dense": 1, "modal": 2}[lh_form])


def osm_query(pb, **opts):
    prob, keep = make_problem(pb)
    opt = make_options(**opts)
    fp = osm_footprint()
    _check(_lib.osm_query(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(fp)))
    return fp.device_bytes, fp.host_bytes


class OsmSolver:
    """Owns one osm_handle.  Tensors: u (ncx+1, ncy+1) complex128, W
    (ncx+1, ncy+1) float64, interface vectors (2(N-1), ncy+1) complex128,
    packed strip vectors (ncx+nsub, ncy+1) complex128, all on the device."""

    def __init__(self, pb, device="cuda:0", **opts):
        self.pb = pb
        self.device = torch.device(device)
        self.ny = pb.ncy + 1
        self.nglob = pb.ncx + 1
        self.lt = pb.ncx + pb.nsub
        self.ntr = 2 * (pb.nsub - 1)
        prob, self._keep = make_problem(pb)
        self._opt = make_options(**opts)
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            h = ctypes.c_void_p()
            _check(_lib.osm_setup(ctypes.byref(prob), ctypes.byref(self._opt),
                                  ctypes.c_void_p(stream), ctypes.byref(h)))
        self.h = h

    def _c(self, status):
        _check(status, self.h)

    def factor(self, W: torch.Tensor):
        assert W.dtype == torch.float64 and W.is_contiguous() and W.numel() == self.nglob * self.ny
        self._c(_lib.osm_factor(self.h, _ptr(W)))

    def factor_rotating(self, n: int):
        self._c(_lib.osm_factor_rotating(self.h, int(n)))

    def step(self, u: torch.Tensor):
        assert u.dtype == torch.complex128 and u.is_contiguous() and u.numel() == self.nglob * self.ny
        st = osm_step_stats()
        status = _lib.osm_step(self.h, _ptr(u), ctypes.byref(st))
        if status != OSM_OK:
            err = OsmError(status, (_lib.osm_last_error(self.h) or b"").decode())
            err.stats = st.as_dict()
            raise err
        return st.as_dict()

    def interface_apply(self, op: int, u, g_in):
        g_out = torch.empty_like(g_in)
        self._c(_lib.osm_interface_apply(self.h, op, _ptr(u), _ptr(g_in), _ptr(g_out)))
        return g_out

    def set_interface_guess(self, g0):
        self._c(_lib.osm_set_interface_guess(self.h, _ptr(g0)))

    def get_interface(self):
        g = torch.empty((self.ntr, self.ny), dtype=torch.complex128, device=self.device)
        self._c(_lib.osm_get_interface(self.h, _ptr(g)))
        return g

    def strip_solve(self, b):
        x = torch.empty_like(b)
        self._c(_lib.osm_strip_solve(self.h, _ptr(b), _ptr(x)))
        return x

    def get_strip_solution(self):
        v = torch.empty((self.lt, self.ny), dtype=torch.complex128, device=self.device)
        self._c(_lib.osm_get_strip_solution(self.h, _ptr(v)))
        return v

    def get_lh_blocks(self):
        b = torch.empty((self.pb.nsub, 4, self.ny, self.ny), dtype=torch.complex128,
                        device=self.device)
        self._c(_lib.osm_get_lh_blocks(self.h, _ptr(b)))
        return b

    def get_factor(self):
        dt = torch.complex64 if self._opt.prec == OSM_C32_REFINE else torch.complex128
        f = torch.empty((self.lt, self.ny, self.ny), dtype=dt, device=self.device)
        self._c(_lib.osm_get_factor(self.h, _ptr(f)))
        return f

    def get_yfactor(self):
        """The y-line-order factor, one (ny, nx_j, nx_j) tensor per strip."""
        nx = [int(c) + 1 for c in self.pb.strip_cells]
        dt = torch.complex64 if self._opt.prec == OSM_C32_REFINE else torch.complex128
        f = torch.empty(sum(self.ny * k * k for k in nx), dtype=dt, device=self.device)
        self._c(_lib.osm_get_yfactor(self.h, _ptr(f)))
        out, o = [], 0
        for k in nx:
            out.append(f[o:o + self.ny * k * k].view(self.ny, k, k))
            o += self.ny * k * k
        return out

    def strip_order(self):
        return "y" if int(_lib.osm_strip_order(self.h)) == 1 else "node"

    def lh_form(self):
        """How L_h is applied: None (not built), "dense", "modal" (dense real
        transforms) or "fft" (the modal form by FFT)."""
        return (None, "dense", "modal", "fft")[int(_lib.osm_lh_form(self.h))]

    def solve_team(self):
        return int(_lib.osm_solve_team(self.h))

    def solve_shape(self):
        return int(_lib.osm_solve_shape(self.h))

    def guess_features(self, g1, g2, g0=None):
        """Network inputs (nsub-1, 9, ny) and, with g0, targets (nsub-1, 4, ny)."""
        T = self.pb.nsub - 1
        x = torch.empty((T, 9, self.ny), dtype=torch.float32, device=self.device)
        t = None
        if g0 is not None:
            t = torch.empty((T, 4, self.ny), dtype=torch.float32, device=self.device)
        self._c(_lib.osm_guess_features(self.h, _ptr(g1), _ptr(g2), _ptr(g0), _ptr(x), _ptr(t)))
        return x, t

    def set_guess_net(self, net):
        self._c(_lib.osm_set_guess_net(self.h, net.h if net is not None else None))
        self._net = net

    def kernel_timing(self, enable: bool):
        """Returns (summed solve-kernel ms, launches) since the last reset."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._c(_lib.osm_kernel_timing(self.h, int(enable), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def kernel_work(self):
        """Algorithmic bytes of the timed solve launches since the last reset."""
        b = ctypes.c_double()
        self._c(_lib.osm_kernel_work(self.h, ctypes.byref(b)))
        return b.value

    def factor_timing(self):
        """(summed ms, launches, algorithmic flops) of the factor's timed
        sweep-update launches since the last kernel_timing reset."""
        ms, f = ctypes.c_double(), ctypes.c_double()
        n = ctypes.c_int64()
        self._c(_lib.osm_factor_timing(self.h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(f)))
        return ms.value, n.value, f.value

    def close(self):
        if self.h:
            _lib.osm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _problem_array(pbs):
    arr = (osm_problem * len(pbs))()
    keep = []
    for i, pb in enumerate(pbs):
        arr[i], k = make_problem(pb)
        keep.append(k)
    return arr, keep


def _ptr_array(ts):
    return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])


def osm_query_batch(pbs, **opts):
    arr, keep = _problem_array(pbs)
    opt = make_options(**opts)
    fp = osm_footprint()
    _check(_lib.osm_query_batch(arr, len(pbs), ctypes.byref(opt), ctypes.byref(fp)))
    return fp.device_bytes, fp.host_bytes


class OsmBatch:
    """Owns one batch handle over independent instances.  Per instance: u
    (ncx+1, ncy+1) complex128 and W (ncx+1, ncy+1) float64 on the device."""

    def __init__(self, pbs, device="cuda:0", **opts):
        self.pbs = list(pbs)
        self.nb = len(self.pbs)
        self.device = torch.device(device)
        arr, self._keep = _problem_array(self.pbs)
        self._opt = make_options(**opts)
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            h = ctypes.c_void_p()
            _check(_lib.osm_setup_batch(arr, self.nb, ctypes.byref(self._opt),
                                        ctypes.c_void_p(stream), ctypes.byref(h)))
        self.h = h

    def _c(self, status):
        _check(status, self.h)

    def _check_fields(self, ts, dtype):
        assert len(ts) == self.nb
        for t, pb in zip(ts, self.pbs):
            assert t.dtype == dtype and t.is_contiguous()
            assert t.numel() == (pb.ncx + 1) * (pb.ncy + 1)

    def factor(self, Ws):
        self._check_fields(Ws, torch.float64)
        self._c(_lib.osm_factor_batch(self.h, _ptr_array(Ws)))

    def step(self, us):
        """Advances every u in place; returns the list of per-instance stats."""
        self._check_fields(us, torch.complex128)
        st = (osm_step_stats * self.nb)()
        status = _lib.osm_step_batch(self.h, _ptr_array(us), st)
        stats = [st[i].as_dict() for i in range(self.nb)]
        if status != OSM_OK:
            err = OsmError(status, (_lib.osm_last_error(self.h) or b"").decode())
            err.stats = stats
            raise err
        return stats

    def tuning(self):
        v = ctypes.c_int32()
        a = ctypes.c_double()
        g = ctypes.c_int32()
        n = ctypes.c_int32()
        self._c(_lib.osm_batch_tuning(self.h, ctypes.byref(v), ctypes.byref(a), ctypes.byref(g),
                                      ctypes.byref(n)))
        return {"variant": v.value, "alpha": a.value, "workgroups": g.value, "items": n.value}

    def kernel_timing(self, enable: bool):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._c(_lib.osm_kernel_timing(self.h, int(enable), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def kernel_work(self):
        b = ctypes.c_double()
        self._c(_lib.osm_kernel_work(self.h, ctypes.byref(b)))
        return b.value

    def close(self):
        if self.h:
            _lib.osm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


NET_NPARAMS = int(_lib.osm_net_nparams())
NET_NOALLOC_MAX_TRACES = 256   # OSM_NET_NOALLOC_MAX_TRACES of include/osm.h


class OsmNet:
    """The interface-guess network (include/osm.h, learned guess)."""

    def __init__(self, max_traces=1024, device="cuda:0"):
        self.device = torch.device(device)
        self.max_traces = max_traces
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            h = ctypes.c_void_p()
            st = _lib.osm_net_create(int(max_traces), ctypes.c_void_p(stream), ctypes.byref(h))
            if st != OSM_OK:
                raise OsmError(st, (_lib.osm_net_last_error(None) or b"").decode())
        self.h = h

    def _c(self, status):
        if status != OSM_OK:
            raise OsmError(status, (_lib.osm_net_last_error(self.h) or b"").decode())

    def set_params(self, theta):
        theta = torch.as_tensor(theta, dtype=torch.float32).to(self.device).contiguous()
        assert theta.numel() == NET_NPARAMS
        self._c(_lib.osm_net_set_params(self.h, _ptr(theta)))

    def get_params(self, rounded=False):
        out = torch.empty(NET_NPARAMS, dtype=torch.float32, device=self.device)
        self._c(_lib.osm_net_get_params(self.h, int(rounded), _ptr(out)))
        return out

    def forward(self, x):
        assert x.dtype == torch.float32 and x.is_contiguous() and x.dim() == 3
        T, C, L = x.shape
        y = torch.empty((T, 4, L), dtype=torch.float32, device=self.device)
        self._c(_lib.osm_net_forward(self.h, _ptr(x), T, L, _ptr(y)))
        return y

    def loss_grad(self, x, t):
        T, _, L = x.shape
        g = torch.empty(NET_NPARAMS, dtype=torch.float32, device=self.device)
        loss = ctypes.c_double()
        self._c(_lib.osm_net_loss_grad(self.h, _ptr(x), _ptr(t), T, L, _ptr(g), ctypes.byref(loss)))
        return loss.value, g

    def loss_grad_noalloc(self, x, t, grad, loss=None):
        """osm_net_loss_grad_noalloc into the caller's device tensors grad
        (NET_NPARAMS float32) and loss (one float64, or None); enqueued on
        the network's stream, not synchronised."""
        T, _, L = x.shape
        self._c(_lib.osm_net_loss_grad_noalloc(self.h, _ptr(x), _ptr(t), T, L, _ptr(grad),
                                               _ptr(loss)))

    def train_step(self, x, t, lr, want_loss=True):
        T, _, L = x.shape
        loss = ctypes.c_double()
        self._c(_lib.osm_net_train_step(self.h, _ptr(x), _ptr(t), T, L, float(lr),
                                        ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def close(self):
        if self.h:
            _lib.osm_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
