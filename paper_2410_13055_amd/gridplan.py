"""ctypes binding of libgridplan (argument marshalling only).

Every step of the dispatch solve, the capacity gradient and the planning
step runs in the HIP library; this module only converts a
``cases.Case`` into the C descriptors of ``include/gridplan.h`` and numpy
arrays into pointers.  It fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgridplan.so")

GP_OK, GP_ENOTCONVERGED = 0, 1
GP_EINVAL, GP_ENOMEM, GP_EHIP, GP_ESTATE = -1, -2, -3, -4

EXPORTS = ("plan_init", "dispatch_solve_batch", "dispatch_grad", "dispatch_objective", "plan_step",
           "plan_set_price_weight",
           "dispatch_get_solution", "dispatch_set_start", "plan_time_sweeps", "plan_tuning",
           "plan_nn_rows", "plan_features", "plan_targets", "plan_start_from_prediction",
           "mlp_init", "mlp_num_params", "mlp_get_params", "mlp_set_params", "mlp_forward", "mlp_forward_noalloc",
           "mlp_loss_grad", "mlp_adam_step", "mlp_fit_scaling", "mlp_get_scaling",
           "mlp_set_scaling", "mlp_time_forward", "mlp_gemm_test", "mlp_free", "mlp_last_error",
           "plan_sizes", "plan_free", "plan_last_error")


class GridplanError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gridplan error {code}: {msg}")
        self.code = code


class NotBuiltError(RuntimeError):
    pass


class gp_network(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_lines", C.c_int32), ("n_gens", C.c_int32),
                ("n_batt", C.c_int32),
                ("line_from", C.POINTER(C.c_int32)), ("line_to", C.POINTER(C.c_int32)),
                ("line_beta", C.POINTER(C.c_double)), ("gen_node", C.POINTER(C.c_int32)),
                ("gen_cost", C.POINTER(C.c_double)), ("gen_emis", C.POINTER(C.c_double)),
                ("batt_node", C.POINTER(C.c_int32)), ("eta_min", C.POINTER(C.c_double)),
                ("eta_max", C.POINTER(C.c_double)), ("n_hvdc", C.c_int32), ("beta_scales", C.c_int32),
                ("gen_ramp", C.POINTER(C.c_double))]


class gp_scenario(C.Structure):
    _fields_ = [("network", C.c_int32), ("T", C.c_int32), ("avail", C.POINTER(C.c_float)),
                ("load", C.POINTER(C.c_float)), ("weight", C.c_double)]


class gp_case_desc(C.Structure):
    _fields_ = [("n_networks", C.c_int32), ("networks", C.POINTER(gp_network)),
                ("n_scenarios", C.c_int32), ("scenarios", C.POINTER(gp_scenario)),
                ("r", C.c_double), ("lambda_u", C.c_double), ("eff", C.c_double),
                ("hours", C.c_double)]


class gp_options(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("check_every", C.c_int32),
                ("block", C.c_int32), ("no_graph", C.c_int32), ("rho0", C.c_double),
                ("verbose", C.c_int32), ("variant", C.c_int32), ("accept_warm", C.c_int32),
                ("stall_pct", C.c_int32), ("reserved", C.c_int32 * 4)]


class gp_solve_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("status", C.c_int32),
                ("start", C.c_int32), ("r_pri", C.c_double), ("r_dual", C.c_double),
                ("r_gap", C.c_double), ("kkt", C.c_double), ("cost", C.c_double),
                ("emis", C.c_double), ("primal_weight", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Load libgridplan.so (raises NotBuiltError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise NotBuiltError(f"{path} not found: run `python -m paper_2410_13055_amd.build`")
    lib = C.CDLL(path)
    P = C.POINTER
    lib.plan_init.argtypes = [P(C.c_void_p), P(gp_case_desc), P(gp_options), C.c_void_p]
    lib.plan_init.restype = C.c_int
    lib.dispatch_solve_batch.argtypes = [C.c_void_p, P(C.c_double), P(C.c_int32), C.c_int32,
                                         C.c_int32, P(C.c_double), P(gp_solve_stats)]
    lib.dispatch_solve_batch.restype = C.c_int
    lib.dispatch_grad.argtypes = [C.c_void_p, P(C.c_double), P(C.c_int32), C.c_int32, C.c_double,
                                  P(C.c_double), P(C.c_double)]
    lib.dispatch_grad.restype = C.c_int
    lib.dispatch_objective.argtypes = [C.c_void_p, P(C.c_double), P(C.c_int32), C.c_int32, C.c_double,
                                       P(C.c_double)]
    lib.dispatch_objective.restype = C.c_int
    lib.plan_set_price_weight.argtypes = [C.c_void_p, C.c_double]
    lib.plan_set_price_weight.restype = C.c_int
    lib.plan_step.argtypes = [C.c_void_p, C.c_double, P(C.c_int32), C.c_int32, P(C.c_double),
                              C.c_double, C.c_int32, P(C.c_double), P(C.c_double), P(C.c_double)]
    lib.plan_step.restype = C.c_int
    lib.dispatch_get_solution.argtypes = [C.c_void_p, C.c_int32, P(C.c_float), P(C.c_double),
                                          P(C.c_int64), P(C.c_int64)]
    lib.dispatch_get_solution.restype = C.c_int
    lib.dispatch_set_start.argtypes = [C.c_void_p, C.c_int32, P(C.c_float), P(C.c_double)]
    lib.dispatch_set_start.restype = C.c_int
    lib.plan_time_sweeps.argtypes = [C.c_void_p, P(C.c_int32), C.c_int32, C.c_int32,
                                     P(C.c_double), P(C.c_double)]
    lib.plan_time_sweeps.restype = C.c_int
    lib.plan_tuning.argtypes = [C.c_void_p, P(C.c_int32), P(C.c_int32), P(C.c_int32), P(C.c_double)]
    lib.plan_tuning.restype = C.c_int
    lib.plan_nn_rows.argtypes = [C.c_void_p, P(C.c_int32), C.c_int32, P(C.c_int64), P(C.c_int32)]
    lib.plan_features.argtypes = [C.c_void_p, P(C.c_double), P(C.c_int32), C.c_int32, C.c_void_p]
    lib.plan_targets.argtypes = [C.c_void_p, P(C.c_int32), C.c_int32, C.c_void_p]
    lib.plan_start_from_prediction.argtypes = [C.c_void_p, P(C.c_double), P(C.c_int32), C.c_int32,
                                               C.c_void_p]
    for f in ("plan_nn_rows", "plan_features", "plan_targets", "plan_start_from_prediction"):
        getattr(lib, f).restype = C.c_int
    lib.mlp_init.argtypes = [P(C.c_void_p), C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
                             C.c_void_p]
    lib.mlp_num_params.argtypes = [C.c_void_p, P(C.c_int64)]
    lib.mlp_get_params.argtypes = [C.c_void_p, P(C.c_float)]
    lib.mlp_set_params.argtypes = [C.c_void_p, P(C.c_float)]
    lib.mlp_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]
    lib.mlp_forward_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, P(C.c_int64)]
    lib.mlp_forward_noalloc.restype = C.c_int
    lib.mlp_loss_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32,
                                  P(C.c_double), P(C.c_float)]
    lib.mlp_adam_step.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_double,
                                  P(C.c_double)]
    lib.mlp_fit_scaling.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32]
    lib.mlp_get_scaling.argtypes = [C.c_void_p, P(C.c_float), P(C.c_float), P(C.c_float), P(C.c_float)]
    lib.mlp_set_scaling.argtypes = [C.c_void_p, P(C.c_float), P(C.c_float), P(C.c_float), P(C.c_float)]
    for f in ("mlp_fit_scaling", "mlp_get_scaling", "mlp_set_scaling"):
        getattr(lib, f).restype = C.c_int
    lib.mlp_time_forward.argtypes = [C.c_void_p, C.c_int64, C.c_int32, P(C.c_double)]
    lib.mlp_time_forward.restype = C.c_int
    lib.mlp_gemm_test.argtypes = [P(C.c_float), P(C.c_float), P(C.c_float), C.c_int32, C.c_int32,
                                  C.c_int32, C.c_int32, C.c_int32]
    for f in ("mlp_init", "mlp_num_params", "mlp_get_params", "mlp_set_params", "mlp_forward",
              "mlp_loss_grad", "mlp_adam_step", "mlp_gemm_test"):
        getattr(lib, f).restype = C.c_int
    lib.mlp_free.argtypes = [C.c_void_p]
    lib.mlp_free.restype = None
    lib.mlp_last_error.argtypes = [C.c_void_p]
    lib.mlp_last_error.restype = C.c_char_p
    lib.plan_sizes.argtypes = [C.c_void_p, P(C.c_int64), P(C.c_int32)]
    lib.plan_sizes.restype = C.c_int
    lib.plan_free.argtypes = [C.c_void_p]
    lib.plan_free.restype = None
    lib.plan_last_error.argtypes = [C.c_void_p]
    lib.plan_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray], ct):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ct))


class _Descriptor:
    """Owns the numpy arrays the C descriptor points into."""

    def __init__(self, case):
        self.keep = []
        nets = (gp_network * len(case.networks))()
        for i, n in enumerate(case.networks):
            arrs = dict(
                line_from=np.ascontiguousarray(n.line_from, np.int32),
                line_to=np.ascontiguousarray(n.line_to, np.int32),
                line_beta=np.ascontiguousarray(n.line_beta, np.float64),
                gen_node=np.ascontiguousarray(n.gen_node, np.int32),
                gen_cost=np.ascontiguousarray(n.gen_cost, np.float64),
                gen_emis=np.ascontiguousarray(n.gen_emis, np.float64),
                batt_node=np.ascontiguousarray(n.batt_node, np.int32),
                eta_min=np.ascontiguousarray(n.eta_min, np.float64),
                eta_max=np.ascontiguousarray(n.eta_max, np.float64),
                gen_ramp=None if getattr(n, "gen_ramp", None) is None
                else np.ascontiguousarray(n.gen_ramp, np.float64))
            self.keep.append(arrs)
            nets[i] = gp_network(
                n.n_nodes, n.n_lines, n.n_gens, n.n_batt,
                _ptr(arrs["line_from"], C.c_int32), _ptr(arrs["line_to"], C.c_int32),
                _ptr(arrs["line_beta"], C.c_double), _ptr(arrs["gen_node"], C.c_int32),
                _ptr(arrs["gen_cost"], C.c_double), _ptr(arrs["gen_emis"], C.c_double),
                _ptr(arrs["batt_node"], C.c_int32), _ptr(arrs["eta_min"], C.c_double),
                _ptr(arrs["eta_max"], C.c_double), int(getattr(n, "n_hvdc", 0)),
                int(getattr(n, "beta_scales", False)), _ptr(arrs["gen_ramp"], C.c_double))
        scs = (gp_scenario * len(case.scenarios))()
        for i, s in enumerate(case.scenarios):
            av = np.ascontiguousarray(s.avail, np.float32)
            ld = np.ascontiguousarray(s.load, np.float32)
            self.keep.append((av, ld))
            scs[i] = gp_scenario(int(s.network), int(s.T), _ptr(av, C.c_float), _ptr(ld, C.c_float),
                                 float(s.weight))
        self.nets, self.scs = nets, scs
        self.desc = gp_case_desc(len(case.networks), nets, len(case.scenarios), scs,
                                 float(case.r), float(case.lambda_u), float(case.eff), float(case.hours))


def options(tol=1e-4, max_iter=0, check_every=0, block=0, no_graph=0, rho0=0.0, verbose=0,
            variant=0, accept_warm=0, stall_pct=0):
    return gp_options(float(tol), int(max_iter), int(check_every), int(block), int(no_graph),
                      float(rho0), int(verbose), int(variant), int(accept_warm), int(stall_pct))


def current_stream():
    """The HIP stream torch is using on the current device (None when torch
    has no GPU)."""
    try:
        import torch
        if torch.cuda.is_available():
            h = torch.cuda.current_stream().cuda_stream
            # the null stream cannot be captured; the library then uses its own
            return C.c_void_p(h) if h else None
    except Exception:
        pass
    return None


class Plan:
    """A plan on the GPU: the case's device layout plus solver state."""

    def __init__(self, case, opts: Optional[gp_options] = None, stream=None):
        self.lib = load()
        self.case = case
        self._desc = _Descriptor(case)
        self.opts = opts if opts is not None else options()
        h = C.c_void_p()
        rc = self.lib.plan_init(C.byref(h), C.byref(self._desc.desc), C.byref(self.opts),
                                stream if stream is not None else None)
        if rc != GP_OK:
            raise GridplanError(rc, self.lib.plan_last_error(None).decode())
        self.h = h
        K = C.c_int64()
        S = C.c_int32()
        self.lib.plan_sizes(self.h, C.byref(K), C.byref(S))
        self.K, self.S = int(K.value), int(S.value)

    def _check(self, rc, allow_nc=True):
        if rc == GP_OK or (allow_nc and rc == GP_ENOTCONVERGED):
            return rc
        raise GridplanError(rc, self.lib.plan_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.plan_free(self.h)
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

    @staticmethod
    def _idx(scen: Sequence[int]):
        return np.ascontiguousarray(np.asarray(scen, dtype=np.int32))

    def solve(self, eta, scen, warm: int = 0):
        """dispatch_solve_batch: returns (cost[nb], [stats dict], rc)."""
        eta = np.ascontiguousarray(eta, np.float64)
        idx = self._idx(scen)
        nb = idx.shape[0]
        cost = np.zeros(nb)
        st = (gp_solve_stats * max(nb, 1))()
        rc = self.lib.dispatch_solve_batch(self.h, _ptr(eta, C.c_double), _ptr(idx, C.c_int32), nb,
                                           int(warm), _ptr(cost, C.c_double), st)
        self._check(rc)
        return cost, [st[i].as_dict() for i in range(nb)], rc

    def grad(self, scen, omega: float = 0.0, eta=None):
        """dispatch_grad: returns (grad[K], weighted mean h, rc).  With eta
        given, the library checks that it is the last solve's."""
        idx = self._idx(scen)
        e = None if eta is None else np.ascontiguousarray(eta, np.float64)
        g = np.zeros(max(self.K, 1))
        h = C.c_double()
        rc = self.lib.dispatch_grad(self.h, _ptr(e, C.c_double), _ptr(idx, C.c_int32), idx.shape[0],
                                    float(omega), _ptr(g, C.c_double), C.byref(h))
        self._check(rc)
        return g[:self.K], float(h.value), rc

    def objective(self, scen, omega: float = 0.0, eta=None):
        """dispatch_objective: the weighted mean planner objective of the
        last solve of ``scen`` (at ``eta`` when given)."""
        idx = self._idx(scen)
        e = None if eta is None else np.ascontiguousarray(eta, np.float64)
        h = C.c_double()
        self._check(self.lib.dispatch_objective(self.h, _ptr(e, C.c_double), _ptr(idx, C.c_int32),
                                                idx.shape[0], float(omega), C.byref(h)), allow_nc=False)
        return float(h.value)

    def set_price_weight(self, lmp: float):
        """plan_set_price_weight: h_s gains lmp * sum pi D."""
        self._check(self.lib.plan_set_price_weight(self.h, float(lmp)), allow_nc=False)

    def step(self, alpha, scen, gamma, eta, omega: float = 0.0, warm: int = 1):
        """plan_step: returns (new eta, phi at the input eta, Delta, rc)."""
        idx = self._idx(scen)
        gam = np.ascontiguousarray(gamma, np.float64)
        e = np.array(eta, dtype=np.float64, copy=True)
        phi = C.c_double()
        delta = np.zeros(max(self.K, 1))
        rc = self.lib.plan_step(self.h, float(alpha), _ptr(idx, C.c_int32), idx.shape[0],
                                _ptr(gam, C.c_double), float(omega), int(warm), _ptr(e, C.c_double),
                                C.byref(phi), _ptr(delta, C.c_double))
        self._check(rc)
        return e, float(phi.value), delta[:self.K], rc

    def solution(self, s: int):
        """(x FP32, y FP64) of scenario s in the canonical orders."""
        nx, ny = C.c_int64(), C.c_int64()
        self._check(self.lib.dispatch_get_solution(self.h, int(s), None, None, C.byref(nx), C.byref(ny)),
                    allow_nc=False)
        x = np.zeros(nx.value, np.float32)
        y = np.zeros(ny.value, np.float64)
        self._check(self.lib.dispatch_get_solution(self.h, int(s), _ptr(x, C.c_float), _ptr(y, C.c_double),
                                                   None, None), allow_nc=False)
        return x, y

    def time_sweeps(self, scen, iters: int = 50):
        """plan_time_sweeps: mean (ms_dual, ms_primal) per launch."""
        idx = self._idx(scen)
        md, mp = C.c_double(), C.c_double()
        self._check(self.lib.plan_time_sweeps(self.h, _ptr(idx, C.c_int32), idx.shape[0], int(iters),
                                              C.byref(md), C.byref(mp)), allow_nc=False)
        return md.value, mp.value

    def tuning(self):
        """(block, variant, check_every, ms table [2 forms x 3 block sizes])."""
        b, v, c = C.c_int32(), C.c_int32(), C.c_int32()
        tab = np.zeros(6)
        self.lib.plan_tuning(self.h, C.byref(b), C.byref(v), C.byref(c), _ptr(tab, C.c_double))
        return int(b.value), int(v.value), int(c.value), tab.reshape(2, 3)

    # ---- learned warm start (device matrices are torch CUDA tensors) ----
    def nn_rows(self, scen):
        idx = self._idx(scen)
        r, t = C.c_int64(), C.c_int32()
        self._check(self.lib.plan_nn_rows(self.h, _ptr(idx, C.c_int32), idx.shape[0], C.byref(r), C.byref(t)),
                    allow_nc=False)
        return int(r.value), int(t.value)

    def features(self, eta, scen, X):
        """Fill the float32 CUDA tensor X [rows, 5T+3] with node features."""
        e = np.ascontiguousarray(eta, np.float64)
        idx = self._idx(scen)
        _check_dev(X)
        self._check(self.lib.plan_features(self.h, _ptr(e, C.c_double), _ptr(idx, C.c_int32), idx.shape[0],
                                           C.c_void_p(X.data_ptr())), allow_nc=False)

    def targets(self, scen, Y):
        """Fill the float32 CUDA tensor Y [rows, 2T] from the stored solutions."""
        idx = self._idx(scen)
        _check_dev(Y)
        self._check(self.lib.plan_targets(self.h, _ptr(idx, C.c_int32), idx.shape[0], C.c_void_p(Y.data_ptr())),
                    allow_nc=False)

    def start_from_prediction(self, eta, scen, P):
        """Seed the next warm solve of the scenarios from a prediction tensor."""
        e = np.ascontiguousarray(eta, np.float64)
        idx = self._idx(scen)
        _check_dev(P)
        self._check(self.lib.plan_start_from_prediction(self.h, _ptr(e, C.c_double), _ptr(idx, C.c_int32),
                                                        idx.shape[0], C.c_void_p(P.data_ptr())), allow_nc=False)

    def set_start(self, s: int, x, y=None):
        x = np.ascontiguousarray(x, np.float32)
        y = None if y is None else np.ascontiguousarray(y, np.float64)
        self._check(self.lib.dispatch_set_start(self.h, int(s), _ptr(x, C.c_float), _ptr(y, C.c_double)),
                    allow_nc=False)


def _check_dev(t):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("expected a contiguous float32 CUDA tensor")


class MLP:
    """The warm-start network in the library (BF16 MFMA GEMMs, Adam)."""

    def __init__(self, n_in, width, hidden_layers, n_out, seed=0, stream=None):
        self.lib = load()
        h = C.c_void_p()
        rc = self.lib.mlp_init(C.byref(h), int(n_in), int(width), int(hidden_layers), int(n_out), int(seed),
                               stream if stream is not None else None)
        if rc != GP_OK:
            raise GridplanError(rc, self.lib.mlp_last_error(None).decode())
        self.h = h
        n = C.c_int64()
        self.lib.mlp_num_params(self.h, C.byref(n))
        self.n_params = int(n.value)
        self.dims = [int(n_in)] + [int(width)] * int(hidden_layers) + [int(n_out)]

    def _check(self, rc):
        if rc != GP_OK:
            raise GridplanError(rc, self.lib.mlp_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.mlp_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        w = np.zeros(self.n_params, np.float32)
        self._check(self.lib.mlp_get_params(self.h, _ptr(w, C.c_float)))
        return w

    def set_params(self, w):
        w = np.ascontiguousarray(w, np.float32)
        assert w.shape == (self.n_params,)
        self._check(self.lib.mlp_set_params(self.h, _ptr(w, C.c_float)))

    @staticmethod
    def _arg(a):
        if isinstance(a, np.ndarray):
            a = np.ascontiguousarray(a, np.float32)
            return a, C.c_void_p(a.ctypes.data), 0
        _check_dev(a)
        return a, C.c_void_p(a.data_ptr()), 1

    def forward(self, X, Y=None):
        Xk, xp, dev = self._arg(X)
        rows = Xk.shape[0]
        if Y is None:
            if dev:
                import torch
                Y = torch.empty((rows, self.dims[-1]), dtype=torch.float32, device=Xk.device)
            else:
                Y = np.zeros((rows, self.dims[-1]), np.float32)
        Yk, yp, ydev = self._arg(Y)
        assert ydev == dev
        self._check(self.lib.mlp_forward(self.h, xp, rows, dev, yp))
        return Y

    def forward_noalloc(self, X, Y):
        """mlp_forward_noalloc on contiguous float32 CUDA tensors X
        [rows x n_in] and Y [rows x n_out]; enqueued on the network's
        stream, no synchronisation.  Returns the library's row limit."""
        _check_dev(X)
        _check_dev(Y)
        cap = C.c_int64()
        self._check(self.lib.mlp_forward_noalloc(self.h, C.c_void_p(X.data_ptr()), int(X.shape[0]),
                                                 C.c_void_p(Y.data_ptr()), C.byref(cap)))
        return int(cap.value)

    def noalloc_rows(self):
        """The row limit of mlp_forward_noalloc for this network (a call with
        NULL buffers fails validation after reporting it)."""
        cap = C.c_int64()
        self.lib.mlp_forward_noalloc(self.h, None, 1, None, C.byref(cap))
        return int(cap.value)

    def loss_grad(self, X, T):
        Xk, xp, dev = self._arg(X)
        Tk, tp, tdev = self._arg(T)
        assert tdev == dev
        loss = C.c_double()
        g = np.zeros(self.n_params, np.float32)
        self._check(self.lib.mlp_loss_grad(self.h, xp, tp, Xk.shape[0], dev, C.byref(loss), _ptr(g, C.c_float)))
        return float(loss.value), g

    def adam_step(self, X, T, lr):
        Xk, xp, dev = self._arg(X)
        Tk, tp, tdev = self._arg(T)
        assert tdev == dev
        loss = C.c_double()
        self._check(self.lib.mlp_adam_step(self.h, xp, tp, Xk.shape[0], dev, float(lr), C.byref(loss)))
        return float(loss.value)


    def fit_scaling(self, X, T):
        """Standardise inputs and targets by the columns' mean and sd."""
        Xk, xp, dev = self._arg(X)
        Tk, tp, tdev = self._arg(T)
        assert tdev == dev
        self._check(self.lib.mlp_fit_scaling(self.h, xp, tp, Xk.shape[0], dev))

    def get_scaling(self):
        """(x_mu, x_sd, y_mu, y_sd) as host float32 arrays."""
        ni, no = self.dims[0], self.dims[-1]
        out = [np.zeros(ni, np.float32), np.zeros(ni, np.float32), np.zeros(no, np.float32),
               np.zeros(no, np.float32)]
        self._check(self.lib.mlp_get_scaling(self.h, *[_ptr(a, C.c_float) for a in out]))
        return tuple(out)

    def set_scaling(self, x_mu, x_sd, y_mu, y_sd):
        arrs = [np.ascontiguousarray(a, np.float32) for a in (x_mu, x_sd, y_mu, y_sd)]
        self._check(self.lib.mlp_set_scaling(self.h, *[_ptr(a, C.c_float) for a in arrs]))

    def time_forward(self, rows, iters=20):
        """Mean ms of one forward pass over rows already loaded (HIP events)."""
        ms = C.c_double()
        self._check(self.lib.mlp_time_forward(self.h, int(rows), int(iters), C.byref(ms)))
        return ms.value

    def flops_per_row(self):
        return 2 * sum(a * b for a, b in zip(self.dims[:-1], self.dims[1:]))


def gemm_test(A, B, M, N, K, ta=False, tb=False):
    """C = op(A) op(B) through the library's BF16 MFMA GEMM (host arrays)."""
    lib = load()
    A = np.ascontiguousarray(A, np.float32)
    B = np.ascontiguousarray(B, np.float32)
    Cm = np.zeros((M, N), np.float32)
    rc = lib.mlp_gemm_test(_ptr(A, C.c_float), _ptr(B, C.c_float), _ptr(Cm, C.c_float), M, N, K, int(ta), int(tb))
    if rc != GP_OK:
        raise GridplanError(rc, lib.mlp_last_error(None).decode())
    return Cm
