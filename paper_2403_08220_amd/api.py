"""Python binding of the DINO-mMALA HIP library: argument marshalling over the C ABI.

Every step of the path runs in the library's kernels; torch supplies device memory
(problem workspaces, stage buffers) and streams.
"""
from __future__ import annotations

import ctypes as ct

import numpy as np

from . import _lib
from ._lib import DinoError, ProblemDesc, check, dptr, fptr, i32ptr, i64ptr  # noqa: F401


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ct.c_void_p(stream.cuda_stream)


def _tp(t):
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else ct.c_void_p(t.data_ptr())


class Context:
    """One GPU: holds the prior/KLE basis and the surrogate network."""

    def __init__(self, device: int = 0):
        self.lib = _lib.load()
        h = ct.c_void_p()
        check(self.lib.dino_ctx_create(device, ct.byref(h)))
        self.h = h
        self.device = device
        self.n = self.r = None
        self.d_out = None
        self.dense = False

    def close(self):
        if self.h:
            check(self.lib.dino_ctx_destroy(self.h))
            self.h = None

    def load_prior(self, n: int, gamma: float, delta: float, r: int):
        check(self.lib.dino_load_prior(self.h, n, gamma, delta, r))
        self.n, self.r = n, r
        self.dense = False

    def load_basis(self, U, lam_dis=None):
        """A dense reduced basis: U (d_m, r) orthonormal columns in whitened KLE coordinates,
        lam_dis (r,) its DIS eigenvalues or None."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        lam = None if lam_dis is None else np.ascontiguousarray(lam_dis, dtype=np.float64)
        check(self.lib.dino_load_basis(self.h, U.shape[1], dptr(U), dptr(lam)))
        self.r = U.shape[1]
        self.dense = True

    @property
    def d_m(self):
        return self.n * self.n

    @property
    def d_perp(self):
        """Length of a complement state: d_m - r (KLE), or d_m (dense basis: the unprojected draw)."""
        return self.d_m if self.dense else self.d_m - self.r

    def read_basis(self):
        dec = np.empty((self.d_m, self.r))
        lam = np.empty(self.r)
        vp = np.empty(self.d_m)
        modes = np.empty((self.r, 2), dtype=np.int32)
        check(self.lib.dino_read_basis(self.h, dptr(dec), dptr(lam), dptr(vp), i32ptr(modes)))
        return dict(dec=dec, lam=lam, var_perp=vp, modes=modes)

    def encode(self, fields, stream=None):
        """Whitened KLE coordinates (x, z_perp) of device fields (n, d_m) in float64."""
        torch = _torch()
        n = fields.shape[0]
        x = torch.empty((n, self.r), dtype=torch.float64, device=fields.device)
        zp = torch.empty((n, self.d_perp), dtype=torch.float64, device=fields.device)
        check(self.lib.dino_encode(self.h, n, _tp(fields), _tp(x), _tp(zp), _stream_handle(stream)))
        return x, zp

    def decode(self, x, z_perp=None, stream=None):
        """Device fields (n, d_m) from whitened coordinates; z_perp None decodes Psi_r x."""
        torch = _torch()
        n = x.shape[0]
        out = torch.empty((n, self.d_m), dtype=torch.float64, device=x.device)
        check(self.lib.dino_decode(self.h, n, _tp(x), _tp(z_perp), _tp(out), _stream_handle(stream)))
        return out

    def load_network(self, layers):
        """layers: list of (kind, W (fan_out x fan_in), b) with kind in linear/act/resid."""
        self._load_layers(self.lib.dino_load_network, layers)

    def load_true_model(self, layers):
        """The true-model stand-in of delayed acceptance (same layer format; its input is the
        first r_T whitened coordinates of the full parameter)."""
        self._load_layers(self.lib.dino_load_true_model, layers, true_model=True)

    def _load_layers(self, fn, layers, true_model=False):
        L = len(layers)
        kinds = np.array([_lib.LAYER_KINDS[k] for k, _, _ in layers], dtype=np.int32)
        Ws = [np.ascontiguousarray(W, dtype=np.float64) for _, W, _ in layers]
        bs = [np.ascontiguousarray(b if b is not None else np.zeros(W.shape[0]), dtype=np.float64)
              for (_, W, b) in layers]
        fo = np.array([W.shape[0] for W in Ws], dtype=np.int32)
        fi = np.array([W.shape[1] for W in Ws], dtype=np.int32)
        Wp = (_lib._D * L)(*[dptr(W) for W in Ws])
        bp = (_lib._D * L)(*[dptr(b) for b in bs])
        check(fn(self.h, L, i32ptr(kinds), i32ptr(fo), i32ptr(fi), Wp, bp))
        if true_model:
            self.true_r_in = int(fi[0])
        else:
            self.d_out = int(fo[-1])


class Problem:
    """n_chains chains of one inverse problem, resident on the device."""

    def __init__(self, ctx: Context, n_chains: int, y, noise_var, dt: float, seed: int = 0, request_id: int = 0,
                 precision: str = "f64", track_complement: bool = True, trace_capacity: int = 0,
                 torch_workspace: bool = True, factorization: str = "primal", method: str = "mmala"):
        self.ctx = ctx
        self.lib = ctx.lib
        y = np.ascontiguousarray(y, dtype=np.float64)
        nv = np.ascontiguousarray(noise_var, dtype=np.float64)
        self.desc = ProblemDesc(n_chains=n_chains, d_y=len(y), precision=_lib.PRECISIONS[precision],
                                track_complement=1 if track_complement else 0, trace_capacity=trace_capacity,
                                factorization=_lib.FACTORIZATIONS[factorization], dt=dt, seed=seed,
                                request_id=request_id, method=_lib.METHODS[method])
        self.method = method
        self.h = None
        nbytes = ct.c_size_t()
        # the library validates the descriptor against the context's prior and network
        check(self.lib.dino_problem_workspace_bytes(ctx.h, ct.byref(self.desc), ct.byref(nbytes)))
        self.C, self.r, self.d_y = n_chains, ctx.r, len(y)
        self.d_perp = ctx.d_perp
        self.track_complement = track_complement
        self.trace_capacity = trace_capacity
        self.dt = dt
        self.ws = None
        ws_ptr = None
        if torch_workspace:
            torch = _torch()
            self.ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=f"cuda:{ctx.device}")
            base = self.ws.data_ptr()
            ws_ptr = ct.c_void_p((base + 255) & ~255)
        h = ct.c_void_p()
        check(self.lib.dino_problem_create(ctx.h, ct.byref(self.desc), dptr(y), dptr(nv), ws_ptr, nbytes.value,
                                           ct.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            check(self.lib.dino_problem_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- chain control ---------------------------------------------------------------
    def init(self, x0=None, z0=None, stream=None):
        x0 = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
        z0 = None if z0 is None else np.ascontiguousarray(z0, dtype=np.float32)
        if x0 is not None:
            assert x0.shape == (self.C, self.r)
        if z0 is not None:
            assert z0.shape == (self.C, self.d_perp)
        check(self.lib.dino_chains_init(self.h, dptr(x0), fptr(z0), _stream_handle(stream)))

    def set_fixed_metric(self, x_map, L_map):
        """LA-pCN: the reduced MAP (r,) and the lower Cholesky factor of I + H there (r, r)."""
        xm = np.ascontiguousarray(x_map, dtype=np.float64)
        Lm = np.ascontiguousarray(L_map, dtype=np.float64)
        assert xm.shape == (self.r,) and Lm.shape == (self.r, self.r)
        check(self.lib.dino_set_fixed_metric(self.h, dptr(xm), dptr(Lm)))

    def step(self, n: int, stream=None):
        check(self.lib.dino_step(self.h, n, _stream_handle(stream)))

    def autotune(self, stream=None) -> int:
        """Time the implementations of this problem's stages and keep the fastest (dino_autotune)."""
        n = np.zeros(1, dtype=np.int32)
        check(self.lib.dino_autotune(self.h, _stream_handle(stream), i32ptr(n)))
        return int(n[0])

    def set_launch_mode(self, mode: str = "graph", steps_per_graph: int = 8):
        """"graph": dino_step replays captured graphs of steps_per_graph transitions; "eager":
        one launch per kernel."""
        check(self.lib.dino_set_launch_mode(self.h, _lib.LAUNCH_MODES[mode], steps_per_graph))

    def set_profiling(self, enable: bool):
        check(self.lib.dino_set_profiling(self.h, 1 if enable else 0))

    def profile(self):
        """Per-stage device time (ms, summed over profiled steps), launches per step, steps."""
        ms = np.zeros(_lib.N_STAGES)
        launches = np.zeros(_lib.N_STAGES, dtype=np.int32)
        steps = np.zeros(1, dtype=np.int64)
        check(self.lib.dino_read_profile(self.h, dptr(ms), i32ptr(launches), i64ptr(steps)))
        names = [self.lib.dino_stage_name(i).decode() for i in range(_lib.N_STAGES)]
        return {n: dict(ms=float(ms[i]), launches=int(launches[i])) for i, n in enumerate(names)}, int(steps[0])

    # --- reads -----------------------------------------------------------------------
    def states(self):
        x = np.empty((self.C, self.r))
        z = np.empty((self.C, self.d_perp), dtype=np.float32) if self.track_complement else None
        check(self.lib.dino_read_states(self.h, dptr(x), fptr(z)))
        return x, z

    def cache(self):
        phi = np.empty(self.C)
        g = np.empty((self.C, self.r))
        L = np.empty((self.C, self.r, self.r))
        check(self.lib.dino_read_cache(self.h, dptr(phi), dptr(g), dptr(L)))
        return phi, g, np.tril(L)

    def diagnostics(self):
        a = np.empty(self.C, dtype=np.int64)
        f = np.empty(self.C, dtype=np.int64)
        s = np.empty(1, dtype=np.int64)
        check(self.lib.dino_read_diagnostics(self.h, i64ptr(a), i64ptr(f), i64ptr(s)))
        return a, f, int(s[0])

    def delayed(self):
        """Delayed acceptance: true misfit of the current states and first-stage passes per chain."""
        phi = np.empty(self.C)
        passes = np.empty(self.C, dtype=np.int64)
        check(self.lib.dino_read_delayed(self.h, dptr(phi), i64ptr(passes)))
        return phi, passes

    def eval_true_misfit(self, z_in, stream=None):
        """True misfit of device rows z_in (n, r_T) float64."""
        torch = _torch()
        out = torch.empty(z_in.shape[0], dtype=torch.float64, device=z_in.device)
        check(self.lib.dino_eval_true_misfit(self.h, z_in.shape[0], _tp(z_in), _tp(out), _stream_handle(stream)))
        return out

    def trace(self):
        n = np.empty(1, dtype=np.int64)
        check(self.lib.dino_read_trace(self.h, None, None, i64ptr(n)))
        k = int(n[0])
        xt = np.empty((k, self.C, self.r), dtype=np.float32)
        pt = np.empty((k, self.C))
        if k:
            check(self.lib.dino_read_trace(self.h, fptr(xt), dptr(pt), i64ptr(n)))
        return xt, pt

    def posterior(self, burn_in: int):
        d_m = self.ctx.d_m
        mean, var = np.empty(d_m), np.empty(d_m)
        xbar, S = np.empty(self.r), np.empty((self.r, self.r))
        check(self.lib.dino_posterior(self.h, burn_in, dptr(mean), dptr(var), dptr(xbar), dptr(S)))
        return mean, var, xbar, S

    def ess(self, burn_in: int):
        e = np.empty(self.r)
        check(self.lib.dino_ess(self.h, burn_in, dptr(e)))
        return e

    # --- stage entry points on device tensors ------------------------------------------
    def eval_geometry(self, x, stream=None, want_H=True):
        torch = _torch()
        n = x.shape[0]
        dev = x.device
        f = torch.empty((n, self.d_y), dtype=torch.float64, device=dev)
        phi = torch.empty(n, dtype=torch.float64, device=dev)
        g = torch.empty((n, self.r), dtype=torch.float64, device=dev)
        H = torch.empty((n, self.r, self.r), dtype=torch.float64, device=dev) if want_H else None
        L = torch.zeros((n, self.r, self.r), dtype=torch.float64, device=dev)
        logdet = torch.empty(n, dtype=torch.float64, device=dev)
        ok = torch.empty(n, dtype=torch.int32, device=dev)
        check(self.lib.dino_eval_geometry(self.h, n, _tp(x), _tp(f), _tp(phi), _tp(g), _tp(H), _tp(L), _tp(logdet),
                                          _tp(ok), _stream_handle(stream)))
        return dict(f=f, phi=phi, g=g, H=H, L=L, logdet=logdet, ok=ok)

    def eval_propose(self, x, g, L, xi, stream=None):
        torch = _torch()
        xp = torch.empty_like(x)
        check(self.lib.dino_eval_propose(self.h, x.shape[0], _tp(x), _tp(g), _tp(L), _tp(xi), _tp(xp),
                                         _stream_handle(stream)))
        return xp

    def eval_log_rho(self, x, cx, xp, cp, stream=None):
        torch = _torch()
        out = torch.empty(x.shape[0], dtype=torch.float64, device=x.device)
        check(self.lib.dino_eval_log_rho(self.h, x.shape[0], _tp(x), _tp(cx["phi"]), _tp(cx["g"]), _tp(cx["L"]),
                                         _tp(cx["logdet"]), _tp(xp), _tp(cp["phi"]), _tp(cp["g"]), _tp(cp["L"]),
                                         _tp(cp["logdet"]), _tp(out), _stream_handle(stream)))
        return out

    def eval_jacobian(self, x, stream=None):
        """Whitened reduced Jacobian (n, d_y, r) at device points x, as the Jacobian stage stores it, in float64."""
        torch = _torch()
        B = torch.empty((x.shape[0], self.d_y, self.r), dtype=torch.float64, device=x.device)
        check(self.lib.dino_eval_jacobian(self.h, x.shape[0], _tp(x), _tp(B), _stream_handle(stream)))
        return B

    def jacobian_ld(self) -> int:
        ld = np.zeros(1, dtype=np.int32)
        check(self.lib.dino_jacobian_ld(self.h, i32ptr(ld)))
        return int(ld[0])

    def jacobian_storage(self, B):
        """Device copy of B (n, d_y, r) in the layout the dual stage entry points take: float64
        rows of r (FP64 problems), or bfloat16 rows padded to dino_jacobian_ld (BF16 and FP8 problems;
        the values are rounded to bfloat16 by torch)."""
        torch = _torch()
        n = B.shape[0]
        ld = self.jacobian_ld()
        if self.desc.precision == _lib.PRECISIONS["f64"]:
            return B.to(torch.float64).contiguous()
        out = torch.zeros((n, self.d_y, ld), dtype=torch.bfloat16, device=B.device)
        out[:, :, : self.r] = B.to(torch.bfloat16)
        return out

    def eval_propose_dual(self, x, g, B, K, logdet, xi, stream=None):
        """Dual-form proposal and forward transition term at device buffers (see dino.h)."""
        torch = _torch()
        xp = torch.empty_like(x)
        lfwd = torch.empty(x.shape[0], dtype=torch.float64, device=x.device)
        check(self.lib.dino_eval_propose_dual(self.h, x.shape[0], _tp(x), _tp(g), _tp(B), _tp(K), _tp(logdet),
                                              _tp(xi), _tp(xp), _tp(lfwd), _stream_handle(stream)))
        return xp, lfwd

    def eval_log_rho_dual(self, x, cx, xp, cp, stream=None):
        """Dual-form log rho^(1); cx, cp: dicts with phi, g, B, K, logdet device tensors."""
        torch = _torch()
        out = torch.empty(x.shape[0], dtype=torch.float64, device=x.device)
        check(self.lib.dino_eval_log_rho_dual(self.h, x.shape[0], _tp(x), _tp(cx["phi"]), _tp(cx["g"]),
                                              _tp(cx["B"]), _tp(cx["K"]), _tp(cx["logdet"]), _tp(xp),
                                              _tp(cp["phi"]), _tp(cp["g"]), _tp(cp["B"]), _tp(cp["K"]),
                                              _tp(cp["logdet"]), _tp(out), _stream_handle(stream)))
        return out

    def eval_normals(self, n: int, stream_id: int, step: int, count: int, stream=None):
        torch = _torch()
        out = torch.empty((n, count), dtype=torch.float64, device=f"cuda:{self.ctx.device}")
        check(self.lib.dino_eval_normals(self.h, n, stream_id, step, count, _tp(out), _stream_handle(stream)))
        return out


def tuning_table():
    """The process-wide tuning table: list of dicts (kind, shape, choice, ms per candidate)."""
    lib = _lib.load()
    n = ct.c_size_t()
    check(lib.dino_tuning_table(None, 0, ct.byref(n)))
    buf = ct.create_string_buffer(n.value + 1)
    check(lib.dino_tuning_table(buf, n.value + 1, ct.byref(n)))
    kinds = {v: k for k, v in _lib.TUNE_KINDS.items()}
    out = []
    for line in buf.value.decode().splitlines():
        f = line.split()
        out.append(dict(kind=kinds[int(f[0])], shape=tuple(int(v) for v in f[1:4]), choice=int(f[4]),
                        ms=[float(v) for v in f[5:]]))
    return out


def tune_set(kind: str, shape, choice: int):
    """Set (choice >= 0) or erase (choice < 0) a tuning-table entry."""
    a, b, c = shape
    check(_lib.load().dino_tune_set(_lib.TUNE_KINDS[kind], a, b, c, choice))


def clear_tuning():
    for e in tuning_table():
        tune_set(e["kind"], e["shape"], -1)


class Server:
    """Continuous-batching server on one GPU (include/dino.h, serving section).

    buckets: list of (d_y, chain slots). Each request runs its own chains (Philox key
    (seed, request_id), prior initial states) and returns its posterior mean field."""

    def __init__(self, ctx: Context, buckets, max_requests: int, steps_per_quantum: int, dt: float,
                 precision: str = "bf16", track_complement: bool = True, hbm_budget_bytes: float = 0.0,
                 factorization: str = "auto"):
        self.ctx = ctx
        self.lib = ctx.lib
        cfg = _lib.ServerCfg()
        cfg.n_buckets = len(buckets)
        for k, (dy, slots) in enumerate(buckets):
            cfg.bucket_dy[k] = dy
            cfg.bucket_slots[k] = slots
        cfg.max_requests = max_requests
        cfg.steps_per_quantum = steps_per_quantum
        cfg.precision = _lib.PRECISIONS[precision]
        cfg.track_complement = 1 if track_complement else 0
        cfg.factorization = _lib.FACTORIZATIONS[factorization]
        cfg.dt = dt
        cfg.hbm_budget_bytes = hbm_budget_bytes
        h = ct.c_void_p()
        check(self.lib.dino_server_create(ctx.h, ct.byref(cfg), ct.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            check(self.lib.dino_server_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def clock(self) -> float:
        t = ct.c_double()
        check(self.lib.dino_server_clock(self.h, ct.byref(t)))
        return t.value

    def submit(self, seed: int, request_id: int, y, noise_var, n_chains: int, n_steps: int, arrival: float = 0.0):
        y = np.ascontiguousarray(y, dtype=np.float64)
        nv = np.ascontiguousarray(noise_var, dtype=np.float64)
        req = _lib.Request(seed=seed, request_id=request_id, d_y=len(y), n_chains=n_chains, n_steps=n_steps,
                           y=dptr(y), noise_var=dptr(nv), arrival=arrival)
        check(self.lib.dino_server_submit(self.h, ct.byref(req)))

    def run(self, until: float = -1.0) -> int:
        n = ct.c_int()
        check(self.lib.dino_server_run(self.h, until, ct.byref(n)))
        return n.value

    def poll(self, max_results: int = 64, with_means: bool = True):
        out = (_lib.Result * max_results)()
        means = np.empty((max_results, self.ctx.d_m)) if with_means else None
        n = ct.c_int()
        check(self.lib.dino_server_poll(self.h, max_results, out, dptr(means), ct.byref(n)))
        res = []
        for k in range(n.value):
            o = out[k]
            d = {f: getattr(o, f) for f, _ in _lib.Result._fields_}
            if with_means:
                d["mean"] = means[k].copy()
            res.append(d)
        return res

    def stats(self):
        a = np.zeros(3, dtype=np.int64)
        check(self.lib.dino_server_stats(self.h, i64ptr(a[0:1]), i64ptr(a[1:2]), i64ptr(a[2:3])))
        return dict(chain_steps=int(a[0]), pending=int(a[1]), live=int(a[2]))
