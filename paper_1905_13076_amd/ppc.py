"""Python binding of the PP-PC library: argument marshalling over the C-ABI.

Every step of the method runs in the HIP library; this module only converts arrays,
passes device pointers of torch CUDA tensors and the current torch stream, and turns
status codes into exceptions.  There is no CPU fallback: without the built library
every call raises.
"""
from __future__ import annotations

import ctypes
from ctypes import byref, c_char_p, c_int32, c_void_p

import numpy as np

from . import _native as nat


class PPCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{nat.STATUS_NAMES.get(code, code)}] {msg}")
        self.code = code


def lib():
    return nat.load()


def _err(h, code):
    msg = lib().ppc_last_error(h)
    return PPCError(code, msg.decode() if msg else "")


def params(**kw) -> nat.Params:
    """ppc_params_default() with keyword overrides (field names of ppc_params)."""
    p = nat.Params()
    lib().ppc_params_default(byref(p))
    names = {f for f, _ in nat.Params._fields_}
    for k, v in kw.items():
        if k not in names:
            raise KeyError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _pd(a):
    return a.ctypes.data_as(nat.PD)


def _pi(a):
    return a.ctypes.data_as(nat.PI)


class _Marshalled:
    """C structs for a problem description, holding the arrays alive."""

    def __init__(self, prob):
        self.xy = _f64(prob.xy).reshape(-1)
        self.tri = _i32(prob.tri).reshape(-1)
        self.dir = _i32(prob.dirichlet)
        self.sigma = _f64(prob.sigma)
        self.mat_id = _i32(prob.mat_id)
        self.js = _f64(prob.js)
        self.order = _i32(prob.orders)
        self.amp = _f64(prob.amps)
        self.phase = _f64(prob.phases)
        models = np.asarray(prob.mat_model)
        par = np.asarray(prob.mat_par, dtype=np.float64).reshape(len(models), 4)
        self.laws = (nat.Law * len(models))()
        for k in range(len(models)):
            self.laws[k].law = int(models[k])
            self.laws[k].nu, self.laws[k].k1, self.laws[k].k2, self.laws[k].k3 = (float(x) for x in par[k])
        self.mesh = nat.Mesh(len(self.xy) // 2, _pd(self.xy), len(self.tri) // 3, _pi(self.tri),
                             len(self.dir), _pi(self.dir))
        self.mat = nat.Material(_pd(self.sigma), _pi(self.mat_id), len(models), self.laws)
        self.exc = nat.Excitation(_pd(self.js), float(prob.f0), len(self.order), _pi(self.order),
                                  _pd(self.amp), _pd(self.phase))


def validate(prob):
    """Host-only check of a problem description: returns (code, message)."""
    m = _Marshalled(prob)
    buf = ctypes.create_string_buffer(512)
    rc = lib().ppc_validate(byref(m.mesh), byref(m.mat), byref(m.exc), buf, 512)
    return rc, buf.value.decode()


def validate_params(p):
    buf = ctypes.create_string_buffer(512)
    rc = lib().ppc_validate_params(byref(p), buf, 512)
    return rc, buf.value.decode()


class Handle:
    def __init__(self, device: int = 0):
        h = c_void_p()
        rc = lib().ppc_create(int(device), byref(h))
        if rc != 0:
            raise _err(None, rc)
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            lib().ppc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream():
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t, shape):
    import torch
    if t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return c_void_p(t.data_ptr())


class Problem:
    """A problem copied to the device (ppc_problem_create)."""

    def __init__(self, handle: Handle, prob):
        self.handle = handle
        m = _Marshalled(prob)
        p = c_void_p()
        rc = lib().ppc_problem_create(handle.h, byref(m.mesh), byref(m.mat), byref(m.exc), byref(p))
        if rc != 0:
            raise _err(handle.h, rc)
        self.p = p
        info = [c_int32() for _ in range(4)]
        lib().ppc_problem_info(p, *(byref(x) for x in info))
        self.n_free, self.nnz, self.n_tri, self.n_nodes = (x.value for x in info)

    def close(self):
        if self.p:
            lib().ppc_problem_destroy(self.p)
            self.p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- PP-PC solve ------------------------------------------------------------------------
    def solve(self, prm, U_init=None, out=None, progress=None):
        """Periodic steady state on the device.  Returns (U [N, n_nodes] CUDA float64,
        eps history (numpy), iterations, stats dict, status).  progress(m, k, eps, active),
        if given, is called after every fine sweep (ppc_params.progress)."""
        import torch
        if progress is not None:
            return _with_progress(prm, progress, lambda: self.solve(prm, U_init, out))
        shape = (prm.N, self.n_nodes)
        if out is None:
            out = torch.empty(shape, dtype=torch.float64, device=f"cuda:{self.handle.device}")
        resid = np.zeros(prm.max_iters + 1, dtype=np.float64)
        iters = c_int32()
        st = nat.Stats()
        ui = _dev_ptr(U_init, shape) if U_init is not None else c_void_p()
        rc = lib().ppc_solve_device(self.handle.h, self.p, byref(prm), ui, _dev_ptr(out, shape),
                                    _pd(resid), byref(iters), byref(st), _stream())
        if rc < 0:
            raise _err(self.handle.h, rc)
        k = iters.value
        return out, resid[: k + 1].copy(), k, st.as_dict(), rc

    def solve_host(self, prm, U_init=None):
        """ppc_solve with host arrays: returns (U numpy, eps, iterations, stats, status)."""
        U = np.zeros((prm.N, self.n_nodes), dtype=np.float64)
        resid = np.zeros(prm.max_iters + 1, dtype=np.float64)
        iters = c_int32()
        st = nat.Stats()
        ui = _f64(U_init) if U_init is not None else None
        rc = lib().ppc_solve(self.handle.h, self.p, byref(prm), _pd(ui) if ui is not None else None,
                             _pd(U), _pd(resid), byref(iters), byref(st))
        if rc < 0:
            raise _err(self.handle.h, rc)
        k = iters.value
        return U, resid[: k + 1].copy(), k, st.as_dict(), rc

    # -- adjoint -------------------------------------------------------------------------------
    def adjoint(self, prm, U_periodic, n_mat, grads=True):
        """Loss and gradients at a periodic state U_periodic ([N, n_nodes], host array or
        CUDA tensor).  Returns (loss, dP/dsigma [n_tri], dP/dk [n_mat, 3], iterations, stats);
        with grads=False only the loss (the gradients are returned as None)."""
        if hasattr(U_periodic, "detach"):
            U_periodic = U_periodic.detach().cpu().numpy()
        Uh = _f64(U_periodic)
        if Uh.shape != (prm.N, self.n_nodes):
            raise ValueError(f"expected shape {(prm.N, self.n_nodes)}")
        loss = np.zeros(1)
        dsig = np.zeros(self.n_tri)
        dk = np.zeros(3 * n_mat)
        iters = c_int32()
        st = nat.Stats()
        rc = lib().ppc_adjoint(self.handle.h, self.p, byref(prm), _pd(Uh), _pd(loss),
                               _pd(dsig) if grads else None, _pd(dk) if grads else None,
                               byref(iters), byref(st))
        if rc < 0:
            raise _err(self.handle.h, rc)
        if not grads:
            return float(loss[0]), None, None, iters.value, st.as_dict()
        return float(loss[0]), dsig, dk.reshape(n_mat, 3), iters.value, st.as_dict()

    # -- single pieces ------------------------------------------------------------------------
    def fine_sweep(self, prm, U):
        """F[n mod N] = F_n(U[n-1]) for all chains (one launch).  U: CUDA [N, n_nodes]."""
        import torch
        shape = (prm.N, self.n_nodes)
        F = torch.empty(shape, dtype=torch.float64, device=U.device)
        newton = np.zeros(prm.N, dtype=np.int32)
        lin = np.zeros(prm.N, dtype=np.int32)
        rc = lib().ppc_fine_sweep_device(self.handle.h, self.p, byref(prm), _dev_ptr(U, shape),
                                         _dev_ptr(F, shape), _pi(newton), _pi(lin), _stream())
        if rc < 0:
            raise _err(self.handle.h, rc)
        return F, newton, lin

    def fine_sweep_noalloc(self, prm, U, F=None):
        """ppc_fine_sweep_noalloc: the fine sweep of fine_sweep() on the library's static
        device scratch (no device allocation by the library).  U, F: CUDA [N, n_nodes]
        (F is allocated here when not given).  Returns (F, newton, lin)."""
        import torch
        shape = (prm.N, self.n_nodes)
        if F is None:
            F = torch.empty(shape, dtype=torch.float64, device=U.device)
        newton = np.zeros(prm.N, dtype=np.int32)
        lin = np.zeros(prm.N, dtype=np.int32)
        rc = lib().ppc_fine_sweep_noalloc(self.handle.h, self.p, byref(prm), _dev_ptr(U, shape),
                                          _dev_ptr(F, shape), _pi(newton), _pi(lin), _stream())
        if rc < 0:
            raise _err(self.handle.h, rc)
        return F, newton, lin

    def fine_counts(self, N):
        """Per-chain counters of the last fine sweep, int32 [N, 8]: status, Newton and PCG
        iterations, largest Newton / PCG count, capped PCG solves, failing step, residual
        evaluations."""
        out = np.zeros((N, 8), dtype=np.int32)
        rc = lib().ppc_fine_counts(self.p, N, _pi(out))
        if rc < 0:
            raise PPCError(rc, "ppc_fine_counts: no sweep with this N on this problem")
        return out

    def time_stepping(self, prm, u_start=None, U_prev=None):
        """ppc_time_stepping_device: classical time stepping period after period until two
        consecutive periods' samples agree to prm.tol_ppc (at most prm.max_iters periods).
        u_start CUDA [n_nodes] or None, U_prev CUDA [N, n_nodes] or None.  Returns (U CUDA
        [N, n_nodes] of the last period, periods stepped, stats dict, status)."""
        import torch
        shape = (prm.N, self.n_nodes)
        out = torch.empty(shape, dtype=torch.float64, device=f"cuda:{self.handle.device}")
        us = _dev_ptr(u_start, (self.n_nodes,)) if u_start is not None else None
        up = _dev_ptr(U_prev, shape) if U_prev is not None else None
        per = np.zeros(1, dtype=np.int32)
        st = nat.Stats()
        rc = lib().ppc_time_stepping_device(self.handle.h, self.p, byref(prm), us, up, _dev_ptr(out, shape),
                                            _pi(per), byref(st), _stream())
        if rc < 0:
            raise _err(self.handle.h, rc)
        return out, int(per[0]), st.as_dict(), rc

    def autotune(self, prm):
        """ppc_autotune: returns (chosen register-row workgroup size or 0, sweep ms at 256,
        512, 1024 threads, NaN where the rows do not fit)."""
        b = np.zeros(1, dtype=np.int32)
        ms = np.zeros(3, dtype=np.float64)
        rc = lib().ppc_autotune(self.handle.h, self.p, byref(prm), _pi(b), _pd(ms))
        if rc < 0:
            raise _err(self.handle.h, rc)
        return int(b[0]), ms

    def coarse_correction(self, prm, U, J):
        """dU solving the cyclic coarse system for jumps J.  CUDA [N, n_nodes] each."""
        import torch
        shape = (prm.N, self.n_nodes)
        dU = torch.empty(shape, dtype=torch.float64, device=U.device)
        cocg = np.zeros(prm.N // 2 + 1, dtype=np.int32)
        rc = lib().ppc_coarse_correction_device(self.handle.h, self.p, byref(prm), _dev_ptr(U, shape),
                                                _dev_ptr(J, shape), _dev_ptr(dU, shape), _pi(cocg),
                                                _stream())
        if rc < 0:
            raise _err(self.handle.h, rc)
        return dU, cocg


class BatchProblem:
    """Several designs copied to the device as one batched problem
    (ppc_problem_create_batch); solve() runs PP-PC on all of them at once."""

    def __init__(self, handle: Handle, probs):
        self.handle = handle
        ms = [_Marshalled(q) for q in probs]
        self._keep = ms
        D = len(ms)
        meshes = (nat.Mesh * D)(*[m.mesh for m in ms])
        mats = (nat.Material * D)(*[m.mat for m in ms])
        excs = (nat.Excitation * D)(*[m.exc for m in ms])
        p = c_void_p()
        rc = lib().ppc_problem_create_batch(handle.h, D, meshes, mats, excs, byref(p))
        if rc != 0:
            raise _err(handle.h, rc)
        self.p = p
        nd = c_int32()
        nn = np.zeros(D, dtype=np.int32)
        nf = np.zeros(D, dtype=np.int32)
        lib().ppc_batch_info(p, byref(nd), _pi(nn), _pi(nf))
        self.n_designs = nd.value
        self.n_nodes = nn
        self.n_free = nf
        self.offsets = np.concatenate([[0], np.cumsum(nn)])

    def close(self):
        if self.p:
            lib().ppc_problem_destroy(self.p)
            self.p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fine_sweep(self, prm, U):
        """One batched fine sweep of every design (ppc_fine_sweep_device on the batch).
        U: flat CUDA float64 [N * sum(n_nodes)] in the batched solve's layout.  Returns
        (F flat, newton [D, N], lin [D, N])."""
        import torch
        total = prm.N * int(self.offsets[-1])
        if U.numel() != total or U.dtype != torch.float64 or not U.is_contiguous() or U.device.type != "cuda":
            raise ValueError(f"expected a contiguous float64 CUDA tensor of {total} values")
        F = torch.empty_like(U)
        newton = np.zeros((self.n_designs, prm.N), dtype=np.int32)
        lin = np.zeros((self.n_designs, prm.N), dtype=np.int32)
        rc = lib().ppc_fine_sweep_device(self.handle.h, self.p, byref(prm), c_void_p(U.data_ptr()),
                                         c_void_p(F.data_ptr()), _pi(newton), _pi(lin), _stream())
        if rc < 0:
            raise _err(self.handle.h, rc)
        return F, newton, lin

    def autotune(self, prm):
        """ppc_autotune by size class: (chosen size per design, ms [D, 3] of its class)."""
        b = np.zeros(self.n_designs, dtype=np.int32)
        ms = np.zeros((self.n_designs, 3), dtype=np.float64)
        rc = lib().ppc_autotune(self.handle.h, self.p, byref(prm), _pi(b), _pd(ms))
        if rc < 0:
            raise _err(self.handle.h, rc)
        return b, ms

    def solve(self, prm, U_init=None, progress=None):
        """Returns (list of per-design U [N, n_nodes_d] CUDA views, eps [D, k+1] numpy,
        iterations per design, stats dict, status).  progress(m, k, eps, active) as for
        Problem.solve (eps: the largest of the iteration's designs)."""
        import torch
        if progress is not None:
            return _with_progress(prm, progress, lambda: self.solve(prm, U_init))
        total = int(self.offsets[-1])
        flat = torch.empty(prm.N * total, dtype=torch.float64, device=f"cuda:{self.handle.device}")
        resid = np.zeros((self.n_designs, prm.max_iters + 1), dtype=np.float64)
        iters = np.zeros(self.n_designs, dtype=np.int32)
        st = nat.Stats()
        if U_init is not None:
            ui = torch.cat([u.reshape(-1) for u in U_init]).contiguous()
            uip = c_void_p(ui.data_ptr())
        else:
            uip = c_void_p()
        rc = lib().ppc_solve_device(self.handle.h, self.p, byref(prm), uip, c_void_p(flat.data_ptr()),
                                    _pd(resid), _pi(iters), byref(st), _stream())
        if rc < 0:
            raise _err(self.handle.h, rc)
        Us = []
        for d in range(self.n_designs):
            a, b = prm.N * int(self.offsets[d]), prm.N * int(self.offsets[d + 1])
            Us.append(flat[a:b].view(prm.N, int(self.n_nodes[d])))
        return Us, resid, iters, st.as_dict(), rc


def _with_progress(prm, fn, call):
    """Run call() with fn(m, k, eps, active) installed as prm.progress, then remove it."""
    cb = nat.PROGRESS(lambda m, k, eps, active, user: fn(m, k, eps, active))
    prm.progress = cb
    try:
        return call()
    finally:
        prm.progress = ctypes.cast(None, nat.PROGRESS)


def problem_params(prob, **kw):
    """Parameters carrying a workload's period and time grid (T, N, m)."""
    return params(T=float(prob.T), N=int(prob.N), m=int(prob.m), **kw)
