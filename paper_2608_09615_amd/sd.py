"""ctypes binding of ``libsd.so`` (argument marshalling only).

Every step of the right-hand side runs in the library's HIP kernels; torch is
used for device memory and the current stream.  If the library is missing the
binding raises: there is no CPU fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsd.so")

SD_OK, SD_EINVAL, SD_ENOMEM, SD_EHIP, SD_ENONFINITE, SD_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
SCHEMES = {"br1": 0, "compact": 1}
PHYSICS = {"diffusion": 0, "pme": 1, "ns": 2}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp32mfma": 3}
INTEGRATORS = {"rk4": 0, "ssprk54": 1}

EXPORTS = ["sd_params_default", "sd_init", "sd_free", "sd_set_stream", "sd_state_size", "sd_rhs",
           "sd_rk_step", "sd_rk_run", "sd_diagnostics", "sd_stable_dt", "sd_set_geometry", "sd_timing", "sd_timing_read",
           "sd_last_error",
           "sd_mlp_param_count", "sd_mlp_work_bytes", "sd_mlp_round_weights", "sd_mlp_forward",
           "sd_mlp_forward_noalloc",
           "sd_mlp_backward", "sd_mse", "sd_mlp_adam", "sd_filter", "sd_closure_set", "sd_closure_rejected",
           "sd_bloch"]


class SDError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libsd error {code}: {msg}")
        self.code = code


class Mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nelem", ctypes.c_int * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3)]


class Params(ctypes.Structure):
    _fields_ = [
        ("physics", ctypes.c_int),
        ("nu", ctypes.c_double),
        ("pme_m", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("Re", ctypes.c_double),
        ("Ma", ctypes.c_double),
        ("Pr", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("u0", ctypes.c_double),
        ("Lref", ctypes.c_double),
        ("sutherland_s", ctypes.c_double),
        ("lambda_over_mu", ctypes.c_double),
        ("entropy_fix", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("ref_state", ctypes.c_int),
        ("eta_ip", ctypes.c_double),
        ("integrator", ctypes.c_int),
    ]


class MlpShape(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int), ("n_hidden", ctypes.c_int), ("n_out", ctypes.c_int)]


class Diag(ctypes.Structure):
    _fields_ = [("ke", ctypes.c_double), ("enstrophy", ctypes.c_double), ("mass", ctypes.c_double),
                ("mom", ctypes.c_double * 3), ("energy", ctypes.c_double), ("umax", ctypes.c_double),
                ("nonfinite", ctypes.c_int), ("smax", ctypes.c_double)]


class BlochCfg(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("scheme", ctypes.c_int), ("J", ctypes.c_double), ("eta_ip", ctypes.c_double)]


_lib = None


def load_library(path=LIB_PATH):
    """Load ``libsd.so`` and declare its C signatures; raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build() "
                          "(there is no CPU fallback)")
    L = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    L.sd_params_default.argtypes = [ctypes.POINTER(Params)]
    L.sd_init.argtypes = [ctypes.POINTER(Mesh), ctypes.c_int, ctypes.c_int, ctypes.POINTER(Params), vp,
                          ctypes.POINTER(vp)]
    L.sd_free.argtypes = [vp]
    L.sd_set_stream.argtypes = [vp, vp]
    L.sd_state_size.argtypes = [vp]
    L.sd_state_size.restype = ctypes.c_longlong
    L.sd_rhs.argtypes = [vp, vp, vp]
    L.sd_rk_step.argtypes = [vp, vp, ctypes.c_double]
    L.sd_rk_run.argtypes = [vp, vp, ctypes.c_double, ctypes.c_longlong]
    L.sd_diagnostics.argtypes = [vp, vp, ctypes.POINTER(Diag)]
    L.sd_stable_dt.argtypes = [vp, vp, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
    L.sd_set_geometry.argtypes = [vp, vp, ctypes.c_int]
    L.sd_timing.argtypes = [vp, ctypes.c_int]
    L.sd_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong)]
    sp = ctypes.POINTER(MlpShape)
    L.sd_mlp_param_count.argtypes = [sp]
    L.sd_mlp_param_count.restype = ctypes.c_longlong
    L.sd_mlp_work_bytes.argtypes = [sp, ctypes.c_int]
    L.sd_mlp_work_bytes.restype = ctypes.c_longlong
    L.sd_mlp_round_weights.argtypes = [sp, vp, vp, vp]
    L.sd_mlp_forward.argtypes = [sp, vp, vp, vp, ctypes.c_int, vp, vp, vp]
    L.sd_mlp_forward_noalloc.argtypes = [sp, vp, vp, vp, ctypes.c_int, vp, vp]
    L.sd_mlp_backward.argtypes = [sp, vp, vp, vp, ctypes.c_int, vp, vp]
    L.sd_mse.argtypes = [vp, vp, vp, ctypes.c_longlong, ctypes.c_int, vp, vp, vp]
    L.sd_mlp_adam.argtypes = [sp, vp, vp, vp, vp, vp, ctypes.c_int, ctypes.c_float, ctypes.c_float,
                              ctypes.c_float, ctypes.c_float, vp]
    L.sd_filter.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp]
    L.sd_closure_set.argtypes = [vp, sp, vp, vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                 ctypes.POINTER(ctypes.c_float), ctypes.c_float]
    L.sd_closure_rejected.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong)]
    L.sd_bloch.argtypes = [ctypes.POINTER(BlochCfg), vp, ctypes.c_longlong, vp, ctypes.c_int, vp, vp, vp, vp, vp]
    L.sd_last_error.argtypes = []
    L.sd_last_error.restype = ctypes.c_char_p
    for f in ("sd_params_default", "sd_init", "sd_free", "sd_set_stream", "sd_rhs", "sd_rk_step", "sd_rk_run",
              "sd_diagnostics", "sd_stable_dt", "sd_set_geometry", "sd_timing", "sd_timing_read",
              "sd_mlp_round_weights",
              "sd_mlp_forward", "sd_mlp_forward_noalloc",
              "sd_mlp_backward", "sd_mse", "sd_mlp_adam", "sd_filter", "sd_closure_set", "sd_closure_rejected",
              "sd_bloch"):
        getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc):
    if rc != SD_OK:
        raise SDError(rc, load_library().sd_last_error().decode())


class SD:
    """One SD discretisation on a periodic Cartesian box.

    ``nelem``: elements per direction (length 1 or 3); ``p``: degree;
    ``scheme``: "compact" or "br1"; ``physics``: "diffusion", "pme" or "ns";
    ``precision``: "fp64", "fp32" or "bf16x3".  Extra keyword arguments set
    the fields of ``sd_params`` (nu, pme_m, gamma, Re, Ma, Pr, eta_ip,
    integrator = "rk4" or "ssprk54", ...).
    """

    def __init__(self, nelem, p, scheme="compact", physics="ns", precision="fp64", lo=None, hi=None,
                 **params):
        import torch
        L = load_library()
        nelem = list(nelem)
        dim = len(nelem)
        if dim not in (1, 3):
            raise ValueError("nelem must have 1 or 3 entries")
        lo = list(lo) if lo is not None else [0.0] * dim
        hi = list(hi) if hi is not None else [1.0] * dim
        m = Mesh(dim, (ctypes.c_int * 3)(*(nelem + [1] * (3 - dim))),
                 (ctypes.c_double * 3)(*(lo + [0.0] * (3 - dim))),
                 (ctypes.c_double * 3)(*(hi + [1.0] * (3 - dim))))
        prm = Params()
        _check(L.sd_params_default(ctypes.byref(prm)))
        prm.physics = PHYSICS[physics]
        prm.precision = PRECISIONS[precision]
        if isinstance(params.get("integrator"), str):
            params["integrator"] = INTEGRATORS[params["integrator"]]
        for k, v in params.items():
            if not hasattr(prm, k):
                raise TypeError(f"unknown parameter {k}")
            setattr(prm, k, v)
        self.dim, self.p, self.n = dim, p, p + 1
        self.nelem = nelem
        self.nv = 5 if physics == "ns" else 1
        self.ne = 1
        for v in nelem:
            self.ne *= v
        self.shape = (self.ne, self.nv) + (self.n,) * dim
        self.params = prm
        self._ctx = ctypes.c_void_p()
        self._graphs = {}
        stream = torch.cuda.current_stream().cuda_stream
        _check(L.sd_init(ctypes.byref(m), p, SCHEMES[scheme], ctypes.byref(prm), ctypes.c_void_p(stream),
                         ctypes.byref(self._ctx)))
        self.size = L.sd_state_size(self._ctx)

    def _stream(self):
        import torch
        _check(load_library().sd_set_stream(self._ctx, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def _check_state(self, u):
        import torch
        if not (isinstance(u, torch.Tensor) and u.is_cuda and u.dtype == torch.float64 and u.is_contiguous()):
            raise TypeError("state must be a contiguous float64 CUDA tensor")
        if u.numel() != self.size:
            raise ValueError(f"state has {u.numel()} values, expected {self.size}")

    def rhs(self, u, out=None):
        import torch
        self._check_state(u)
        if out is None:
            out = torch.empty_like(u)
        self._check_state(out)
        self._stream()
        _check(load_library().sd_rhs(self._ctx, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(out.data_ptr())))
        return out

    def rk_step(self, u, dt):
        self._check_state(u)
        self._stream()
        _check(load_library().sd_rk_step(self._ctx, ctypes.c_void_p(u.data_ptr()), float(dt)))
        return u

    def rk_run(self, u, dt, nsteps):
        """``nsteps`` steps of size ``dt`` on ``u`` in place (sd_rk_run: one
        launch for the whole run of a small one-dimensional FP64 problem,
        otherwise the steps one by one; the same state either way, to the
        last bit of a value)."""
        self._check_state(u)
        self._stream()
        _check(load_library().sd_rk_run(self._ctx, ctypes.c_void_p(u.data_ptr()), float(dt), int(nsteps)))
        return u

    def rk_steps(self, u, dt, nsteps, graph_steps=0):
        """``nsteps`` steps of sd_rk_step on ``u`` (in place).  With
        ``graph_steps`` > 0 the launches of ``graph_steps`` consecutive steps
        are captured once into a HIP graph on a side stream and the graph is
        replayed on the current stream (the first step runs eagerly, so that
        every buffer the steps use exists before the capture; a remainder
        runs eagerly too).  The results are those of the eager steps: the
        graph replays the same kernels on the same buffers.  The graph is
        kept with the context for later calls with the same state, step and
        length; keep timing() off while steps are captured."""
        import torch
        nsteps = int(nsteps)
        if graph_steps <= 0 or nsteps <= graph_steps:
            for _ in range(nsteps):
                self.rk_step(u, dt)
            return u
        self.rk_step(u, dt)
        left = nsteps - 1
        if left < graph_steps:
            for _ in range(left):
                self.rk_step(u, dt)
            return u
        # one graph per (state, step, graph length), kept with the context so
        # that later calls replay it and no replay outlives its graph
        key = (u.data_ptr(), float(dt), int(graph_steps))
        graph = self._graphs.get(key)
        if graph is None:
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                with torch.cuda.graph(graph, stream=side):
                    for _ in range(graph_steps):
                        self.rk_step(u, dt)
            torch.cuda.current_stream().wait_stream(side)
            self._graphs[key] = graph
        for _ in range(left // graph_steps):
            graph.replay()
        for _ in range(left % graph_steps):
            self.rk_step(u, dt)
        # the context's stream back to the one the replays ran on (its later
        # calls, and sd_free's wait, follow them)
        self._stream()
        return u

    def diagnostics(self, u, raise_nonfinite=False):
        self._check_state(u)
        self._stream()
        d = Diag()
        rc = load_library().sd_diagnostics(self._ctx, ctypes.c_void_p(u.data_ptr()), ctypes.byref(d))
        if rc != SD_OK and not (rc == SD_ENONFINITE and not raise_nonfinite):
            _check(rc)
        return {"ke": d.ke, "enstrophy": d.enstrophy, "mass": d.mass, "mom": list(d.mom),
                "energy": d.energy, "umax": d.umax, "nonfinite": bool(d.nonfinite), "smax": d.smax}

    def set_geometry(self, nodes):
        """Curvilinear elements (3-D diffusion or Navier-Stokes, FP64 or FP32): nodes[e][c][b][a][3],
        q + 1 equispaced nodes per direction of every element (q = 1 or 2)."""
        import numpy as np
        nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        q = nodes.shape[1] - 1
        if nodes.ndim != 5 or nodes.shape[1:] != (q + 1, q + 1, q + 1, 3) or nodes.shape[0] != self.ne:
            raise ValueError(f"nodes must have shape [{self.ne}, q+1, q+1, q+1, 3]")
        _check(load_library().sd_set_geometry(self._ctx, nodes.ctypes.data_as(ctypes.c_void_p), q))

    def stable_dt(self, u, cfl=0.3):
        """cfl * min h / ((p + 1) max(|u| + c)) for the state u (sd_stable_dt)."""
        self._check_state(u)
        self._stream()
        dt = ctypes.c_double()
        _check(load_library().sd_stable_dt(self._ctx, ctypes.c_void_p(u.data_ptr()), cfl, ctypes.byref(dt)))
        return dt.value

    def timing(self, enable=True):
        """Start (or stop) recording HIP events around every RHS evaluation."""
        _check(load_library().sd_timing(self._ctx, 1 if enable else 0))

    def timing_read(self):
        """(total ms, number of timed RHS evaluations) since timing() began."""
        ms = ctypes.c_double()
        cnt = ctypes.c_longlong()
        _check(load_library().sd_timing_read(self._ctx, ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value

    def closure_set(self, mlp, in_shift=None, in_scale=None, out_scale=None, max_ratio=1.0):
        """Add the network ``mlp`` (an :class:`Mlp`) as a per-element closure;
        ``mlp=None`` switches it off.  An element's correction is discarded
        when non-finite or, with ``max_ratio`` > 0, larger in max norm than
        ``max_ratio`` times its right-hand side."""
        f5 = ctypes.c_float * 5
        if mlp is None:
            _check(load_library().sd_closure_set(self._ctx, None, None, None, None, None, None, 0.0))
            self._closure = None
            return
        self._closure = mlp
        _check(load_library().sd_closure_set(self._ctx, ctypes.byref(mlp.shape), _ptr(mlp.P), _ptr(mlp.Wb),
                                             f5(*in_shift), f5(*in_scale), f5(*out_scale), float(max_ratio)))

    def closure_rejected(self):
        n = ctypes.c_longlong()
        _check(load_library().sd_closure_rejected(self._ctx, ctypes.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            if getattr(self, "_graphs", None):
                # captured steps reference the context's buffers: let every
                # replay finish, then drop the graphs before the buffers go
                import torch
                torch.cuda.synchronize()
                self._graphs.clear()
            load_library().sd_free(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Mlp:
    """Closure network n_in -> n_hidden -> n_hidden -> n_out (GELU) with FP32
    master parameters ``P`` and their BF16 copy ``Wb`` (device tensors)."""

    def __init__(self, n_in, n_hidden, n_out, P=None):
        import torch
        self.shape = MlpShape(n_in, n_hidden, n_out)
        L = load_library()
        self.nparams = L.sd_mlp_param_count(ctypes.byref(self.shape))
        if self.nparams < 0:
            raise SDError(SD_EINVAL, L.sd_last_error().decode())
        self.P = torch.zeros(self.nparams, dtype=torch.float32, device="cuda") if P is None else P
        self.Wb = torch.zeros(self.nparams, dtype=torch.int16, device="cuda")
        self.m = torch.zeros_like(self.P)
        self.v = torch.zeros_like(self.P)
        self.grad = torch.zeros_like(self.P)
        self.step = 0
        self._work = None
        self._wbatch = 0
        self.round_weights()

    def round_weights(self):
        _check(load_library().sd_mlp_round_weights(ctypes.byref(self.shape), _ptr(self.P), _ptr(self.Wb),
                                                   _stream()))

    def work(self, batch):
        import torch
        if batch > self._wbatch:
            nb = load_library().sd_mlp_work_bytes(ctypes.byref(self.shape), batch)
            self._work = torch.empty(nb, dtype=torch.uint8, device="cuda")
            self._wbatch = batch
        return self._work

    def forward(self, X, Y=None):
        import torch
        B = X.shape[0]
        if Y is None:
            Y = torch.empty((B, self.shape.n_out), dtype=torch.float32, device="cuda")
        _check(load_library().sd_mlp_forward(ctypes.byref(self.shape), _ptr(self.P), _ptr(self.Wb), _ptr(X), B,
                                             _ptr(Y), _ptr(self.work(B)), _stream()))
        return Y

    def forward_noalloc(self, X, Y):
        """Forward pass into the caller's ``Y`` with the library's static
        activation workspace (no device allocation by the library)."""
        _check(load_library().sd_mlp_forward_noalloc(ctypes.byref(self.shape), _ptr(self.P), _ptr(self.Wb), _ptr(X),
                                                     X.shape[0], _ptr(Y), _stream()))
        return Y

    def backward(self, dY):
        B = dY.shape[0]
        _check(load_library().sd_mlp_backward(ctypes.byref(self.shape), _ptr(self.Wb), _ptr(self.work(B)),
                                              _ptr(dY), B, _ptr(self.grad), _stream()))
        return self.grad

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        _check(load_library().sd_mlp_adam(ctypes.byref(self.shape), _ptr(self.P), _ptr(self.Wb), _ptr(self.grad),
                                          _ptr(self.m), _ptr(self.v), self.step, lr, beta1, beta2, eps,
                                          _stream()))


def mse(Y, T, dY, loss, w=None):
    """Row-weighted MSE of Y [rows, cols] against T: dY = 2 w (Y - T) / n and
    the loss into a one-element FP64 device tensor (``loss`` None: dY only);
    ``w`` [rows] FP32 or None."""
    if Y.dim() != 2:
        raise ValueError("Y must be [rows, cols]")
    if w is not None and w.numel() != Y.shape[0]:
        raise ValueError("w must hold one weight per row")
    _check(load_library().sd_mse(_ptr(Y), _ptr(T), None if w is None else _ptr(w), Y.shape[0], Y.shape[1],
                                 _ptr(dY), None if loss is None else _ptr(loss), _stream()))


def filter_state(fine, nel_fine, ratio, p, nv):
    """L2 projection of a fine state onto the coarse elements (device tensors)."""
    import torch
    nec = 1
    for d in range(3):
        nec *= nel_fine[d] // ratio
    out = torch.empty((nec, nv) + (p + 1,) * 3, dtype=torch.float64, device="cuda")
    nel = (ctypes.c_int * 3)(*nel_fine)
    _check(load_library().sd_filter(_ptr(fine), nel, ratio, p, nv, _ptr(out), _stream()))
    return out


def bloch(p, scheme, theta, t=None, J=0.5, eta_ip=0.0, matrices=True, eigs=True):
    """Batched Bloch analysis of the 1-D diffusion operator (sd_bloch).

    theta: CUDA float64 tensor of wavenumbers per element; t: CUDA float64
    tensor of times for the combined mode (None: skip).  Returns complex128
    tensors "B" [ntheta, p+1, p+1], "lam" [ntheta, p+1] and, with t, "G" and
    "omega" [ntheta, nt]."""
    import torch
    if theta.dtype != torch.float64 or not theta.is_cuda or not theta.is_contiguous():
        raise ValueError("theta must be a contiguous CUDA float64 tensor")
    if t is not None and (t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous()):
        raise ValueError("t must be a contiguous CUDA float64 tensor")
    n, nth = p + 1, theta.numel()
    nt = 0 if t is None else t.numel()
    dev = theta.device
    out = {}
    B = torch.empty((nth, n, n, 2), dtype=torch.float64, device=dev) if matrices else None
    lam = torch.empty((nth, n, 2), dtype=torch.float64, device=dev) if eigs else None
    G = torch.empty((nth, nt, 2), dtype=torch.float64, device=dev) if nt else None
    om = torch.empty((nth, nt, 2), dtype=torch.float64, device=dev) if nt else None
    cfg = BlochCfg(p, SCHEMES[scheme], J, eta_ip)
    ptr = lambda x: ctypes.c_void_p(x.data_ptr()) if x is not None else None
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    _check(load_library().sd_bloch(ctypes.byref(cfg), ptr(theta), nth, ptr(t), nt, ptr(B), ptr(lam), ptr(G),
                                   ptr(om), stream))
    for k, x in (("B", B), ("lam", lam), ("G", G), ("omega", om)):
        if x is not None:
            out[k] = torch.view_as_complex(x)
    return out
