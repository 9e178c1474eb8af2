"""MI355X-native inexact All-Floating IETI (AF-IETI) with Fast
Diagonalization local solvers for multi-patch isogeometric compressible
linear elasticity (Bosy, Montardini, Sangalli, Tani, arXiv 2001.09626).

Thin Python binding of the C ABI in ``include/afieti.h``: this module only
marshals arguments; all setup and every step of the solve run in
``libafieti.so`` (C++ host setup, HIP kernels for gfx950).  Device vectors
are torch float64 CUDA tensors used as plain memory, and work is enqueued on
torch's current stream.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _native as N

__all__ = ["Solver", "AfietiError", "to_c_problems", "AfietiSolve", "mass_norm_loss"]


class AfietiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{N.ERRORS.get(code, code)}: {msg}")
        self.code = code


def _field_cb(fn, dim):
    """C callback over a batch of points for a Python f(x[n, dim]) -> [n, dim]."""
    def cb(n, x, out, ctx):
        X = np.ctypeslib.as_array(x, shape=(n, dim))
        np.ctypeslib.as_array(out, shape=(n, dim))[:] = np.asarray(fn(X.copy()), dtype=np.float64).reshape(n, dim)
    return N.FIELD_FN(cb)


def _traction_cb(fn, dim):
    """C callback for a Python g(x[n, dim], normal[n, dim]) -> [n, dim]."""
    def cb(n, x, nrm, out, ctx):
        X = np.ctypeslib.as_array(x, shape=(n, dim)).copy()
        Nv = np.ctypeslib.as_array(nrm, shape=(n, dim)).copy()
        np.ctypeslib.as_array(out, shape=(n, dim))[:] = np.asarray(fn(X, Nv), dtype=np.float64).reshape(n, dim)
    return N.TRACTION_FN(cb)


def to_c_problems(problems):
    """Convert ``workloads`` problem dictionaries into the C structs; returns
    (array, keepalive).  Optional entries: a patch's ``knots`` (explicit
    open knot vectors per direction) and ``ctrl`` (explicit control net,
    shape (n_d, .., n_1, dim), in place of ``corners``), a problem's ``body_force(x)``,
    ``traction(x, normal)`` and ``dirichlet(x)`` callables (arrays of
    points in, arrays of values out), and ``interfaces``: rows (patch_a,
    face_a, patch_b, face_b, orient) gluing only the listed faces (orient
    -1: from the corners)."""
    if isinstance(problems, dict):
        problems = [problems]
    arr = (N.Problem * len(problems))()
    keep = []
    for j, pr in enumerate(problems):
        dim = int(pr["dim"])
        pats = (N.Patch * len(pr["patches"]))()
        for k, pd in enumerate(pr["patches"]):
            P = pats[k]
            P.p = int(pd["p"])
            P.reg = int(pd["reg"])
            for l in range(3):
                P.n_el[l] = int(pd["n_el"][l]) if l < dim else 1
            if pd.get("ctrl") is not None:
                # explicit control net (n_d, .., n_1, dim) -> [node][3]
                X = np.asarray(pd["ctrl"], dtype=np.float64).reshape(-1, dim)
                X3 = np.zeros((len(X), 3))
                X3[:, :dim] = X
                X3 = np.ascontiguousarray(X3)
                keep.append(X3)
                P.ctrl = X3.ctypes.data_as(C.POINTER(C.c_double))
            else:
                cs = np.asarray(pd["corners"], dtype=float)
                for c in range(2 ** dim):
                    for x in range(dim):
                        P.corners[3 * c + x] = float(cs[c, x])
            P.lam = float(pd["lam"])
            P.mu = float(pd["mu"])
            for f in range(2 * dim):
                P.face_bc[f] = int(pd["bc"][f])
            if pd.get("knots") is not None:
                for l in range(dim):
                    kv = np.ascontiguousarray(np.asarray(pd["knots"][l], dtype=np.float64))
                    keep.append(kv)
                    P.knots[l] = kv.ctypes.data_as(C.POINTER(C.c_double))
                    P.n_knots[l] = len(kv)
        modes = (N.LoadMode * max(1, len(pr["load"])))()
        for m, (comp, amp, k, ph) in enumerate(pr["load"]):
            modes[m].comp = int(comp)
            modes[m].amp = float(amp)
            for d in range(dim):
                modes[m].k[d] = int(k[d])
                modes[m].phase[d] = float(ph[d])
        keep += [pats, modes]
        arr[j].dim = dim
        arr[j].n_patches = len(pr["patches"])
        arr[j].patches = pats
        arr[j].n_load_modes = len(pr["load"])
        arr[j].load_modes = modes
        if pr.get("interfaces") is not None:
            # explicit interface list: rows (patch_a, face_a, patch_b, face_b, orient)
            itf = np.ascontiguousarray(np.asarray(pr["interfaces"], dtype=np.int32).reshape(-1, 5))
            keep.append(itf)
            arr[j].n_interfaces = len(itf)
            if len(itf):
                arr[j].interfaces = itf.ctypes.data_as(C.POINTER(C.c_int))
        for key, make in (("body_force", _field_cb), ("traction", _traction_cb), ("dirichlet", _field_cb)):
            if pr.get(key) is not None:
                cb = make(pr[key], dim)
                keep.append(cb)
                setattr(arr[j], key, cb)
    return arr, keep


def _ptr(t):
    return C.c_void_p(0) if t is None else C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Solver:
    """One handle over one or more independent problems."""

    def __init__(self, problems, tol=1e-8, maxit=5000, fd_precision="fp64", ps_variant="nr",
                 check_every=12, host_only=False, use_graph=True, stiffness="auto", fd_tune=-1,
                 ps_weight=1.0, precond="fd", allocator=None):
        """``allocator="torch"``: the handle's device memory comes from
        torch's caching allocator (on the current device and stream)
        instead of hipMalloc, and goes back to it at ``close``."""
        L = N.lib()
        self._L = L
        arr, keep = to_c_problems(problems)
        opt = N.Options()
        L.afieti_default_options(C.byref(opt))
        opt.tol = tol
        opt.maxit = maxit
        opt.fd_precision = N.FD_PRECISION[fd_precision]
        opt.ps_variant = N.PS_VARIANT[ps_variant]
        opt.check_every = check_every
        opt.host_only = 1 if host_only else 0
        opt.use_graph = 1 if use_graph else 0
        opt.stiffness = N.STIFFNESS[stiffness]
        opt.fd_tune = int(fd_tune)
        opt.ps_weight = float(ps_weight)
        opt.precond = N.PRECOND[precond]
        self._alloc_cbs = None
        self._alloc_error = None
        if allocator == "torch":
            import torch
            dev = torch.cuda.current_device()
            alloc_stream = int(torch.cuda.current_stream(dev).cuda_stream)

            def _alloc(nbytes, ctx):
                try:
                    return int(torch.cuda.caching_allocator_alloc(int(nbytes), dev, alloc_stream))
                except Exception as e:  # an exception cannot cross the C boundary: report NULL
                    self._alloc_error = f"{type(e).__name__}: {e}"
                    return 0

            def _free(ptr, nbytes, ctx):
                try:
                    torch.cuda.caching_allocator_delete(ptr)
                except Exception:
                    pass

            self._alloc_cbs = (N.DEV_ALLOC_FN(_alloc), N.DEV_FREE_FN(_free))
            opt.dev_alloc = C.cast(self._alloc_cbs[0], C.c_void_p)
            opt.dev_free = C.cast(self._alloc_cbs[1], C.c_void_p)
        elif allocator is not None:
            raise ValueError(f"unknown allocator {allocator!r}")
        self.host_only = host_only
        h = C.c_void_p()
        stream = C.c_void_p(0) if host_only else _stream()
        code = L.afieti_setup(arr, len(arr), C.byref(opt), stream, C.byref(h))
        if code != N.OK:
            msg = L.afieti_last_error(None).decode()
            if self._alloc_error:
                msg += f" ({self._alloc_error})"
            raise AfietiError(code, msg)
        self._h = h
        info = N.Info()
        L.afieti_get_info(h, C.byref(info))
        self.n_dof = info.n_dof
        self.n_c = info.n_c
        self.n_problems = info.n_problems
        self.n_patches = info.n_patches_total
        self.device_bytes = info.device_bytes
        self.stiffness_bytes = info.stiffness_bytes
        dof = (C.c_int64 * (self.n_patches + 1))()
        coff = (C.c_int64 * (self.n_problems + 1))()
        L.afieti_get_offsets(h, dof, coff)
        self.dof_offsets = np.array(dof[:], dtype=np.int64)
        self.c_offsets = np.array(coff[:], dtype=np.int64)
        probs = [problems] if isinstance(problems, dict) else list(problems)
        self.n_load_modes_total = sum(len(p["load"]) for p in probs)
        self.lame = np.array([[pd["lam"], pd["mu"]] for p in probs for pd in p["patches"]], dtype=np.float64)
        self.amps = np.array([m[1] for p in probs for m in p["load"]], dtype=np.float64)
        self.param_version = 0

    # ----------------------------------------------------------- helpers
    def _check(self, code, allow=(N.OK,)):
        if code not in allow:
            raise AfietiError(code, self._L.afieti_last_error(self._h).decode())
        return code

    def _new(self, n):
        import torch
        return torch.empty(n, dtype=torch.float64, device="cuda")

    def close(self):
        if getattr(self, "_h", None):
            self._L.afieti_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- calls
    def apply_fd(self, r, z=None):
        z = self._new(self.n_dof) if z is None else z
        self._check(self._L.afieti_apply_fd(self._h, _ptr(r), _ptr(z), _stream()))
        return z

    def apply(self, op, x=None, y=None):
        n_out = {"B": self.n_c, "P_chi": self.n_c, "P_S": self.n_c,
                 "prec": self.n_dof + self.n_c, "saddle": self.n_dof + self.n_c}.get(op, self.n_dof)
        y = self._new(n_out) if y is None else y
        self._check(self._L.afieti_apply(self._h, N.OPS[op], _ptr(x), _ptr(y), _stream()))
        return y

    def solve(self, rhs=None, u=None, lam=None, want_lambda=True, allow_not_converged=False):
        u = self._new(self.n_dof) if u is None else u
        if want_lambda and lam is None:
            lam = self._new(self.n_c)
        st = N.Stats()
        allow = (N.OK, N.NOT_CONVERGED) if allow_not_converged else (N.OK,)
        code = self._check(self._L.afieti_solve(self._h, _ptr(rhs), _ptr(u), _ptr(lam),
                                                C.byref(st), _stream()), allow)
        stats = dict(iterations=st.iterations, converged=bool(st.converged),
                     rel_residual=st.rel_residual, ms=st.ms_solve, code=code)
        return u, lam, stats

    def problem_stats(self):
        """Per-problem (iterations, |eta|/gamma_1, status) of the last solve;
        status 1 converged, 2 breakdown, 3 maxit."""
        its = (C.c_int * self.n_problems)()
        rel = (C.c_double * self.n_problems)()
        sta = (C.c_int * self.n_problems)()
        self._check(self._L.afieti_get_problem_stats(self._h, its, rel, sta))
        return np.array(its[:]), np.array(rel[:]), np.array(sta[:])

    def set_parameters(self, lame=None, amps=None):
        """New per-patch (lambda, mu) (array (n_patches, 2)) and/or load
        amplitudes (one per load mode, problems stacked)."""
        lp = ap = None
        if lame is not None:
            lame = np.ascontiguousarray(np.asarray(lame, dtype=np.float64).reshape(self.n_patches, 2))
            lp = lame.ctypes.data_as(C.POINTER(C.c_double))
        if amps is not None:
            amps = np.ascontiguousarray(np.asarray(amps, dtype=np.float64).reshape(self.n_load_modes_total))
            ap = amps.ctypes.data_as(C.POINTER(C.c_double))
        self._check(self._L.afieti_set_parameters(self._h, lp, ap, _stream()))
        if lame is not None:
            self.lame = lame.copy()
        if amps is not None:
            self.amps = amps.copy()
        self.param_version += 1

    def solve_adjoint(self, dJdu, u, psi=None, allow_not_converged=False, load_vectors=None):
        """psi = adjoint state; returns (psi, dJ/dlambda[n_patches],
        dJ/dmu[n_patches], dJ/damp[n_modes], iterations), and with
        ``load_vectors`` (device tensor [m, n_dof]) also dJ/dc[m] for a load
        sum_j c_j F_j as a sixth entry."""
        psi = self._new(self.n_dof) if psi is None else psi
        dl = (C.c_double * (2 * self.n_patches))()
        n_modes = self.n_load_modes_total
        da = (C.c_double * max(1, n_modes))()
        m = 0 if load_vectors is None else int(load_vectors.shape[0])
        dv = (C.c_double * max(1, m))()
        lvt = None if load_vectors is None else load_vectors.contiguous()
        lv = C.c_void_p(0) if lvt is None else C.c_void_p(lvt.data_ptr())
        st = N.Stats()
        allow = (N.OK, N.NOT_CONVERGED) if allow_not_converged else (N.OK,)
        self._check(self._L.afieti_solve_adjoint(self._h, _ptr(dJdu), _ptr(u), _ptr(psi), dl, da, m, lv, dv,
                                                 C.byref(st), _stream()), allow)
        dl = np.array(dl[:]).reshape(-1, 2)
        out = (psi, dl[:, 0], dl[:, 1], np.array(da[:n_modes]), st.iterations)
        return out + (np.array(dv[:m]),) if load_vectors is not None else out

    # ---------------------------------------------------------- exports
    def export(self, what):
        n = self._L.afieti_export_size(self._h, N.EXPORT[what])
        if n < 0:
            raise AfietiError(-1, "bad export")
        if what == "B":
            buf = np.zeros(n // 8, dtype=np.int64)
        else:
            buf = np.zeros(n // 8, dtype=np.float64)
        self._check(self._L.afieti_export(self._h, N.EXPORT[what], buf.ctypes.data_as(C.c_void_p), n))
        if what == "B":
            return buf.reshape(-1, 3)
        if what == "geo_scale":
            return buf.reshape(2, -1)
        if what == "glue":
            return buf.reshape(-1, 3)
        if what == "GtG":
            m = int(round(np.sqrt(len(buf))))
            return buf.reshape(m, m)
        return buf


def _autograd():
    import torch

    class _AfietiSolve(torch.autograd.Function):
        """u = AF-IETI solution for per-patch Lame parameters ``lame``
        (n_patches x 2: lambda, mu) and load amplitudes ``amps``.  The
        backward pass is one adjoint AF-IETI solve with right-hand side
        dJ/du (the saddle operator is symmetric) plus the per-patch
        strain-energy contractions; Krylov iterates are not stored."""

        @staticmethod
        def forward(ctx, lame, amps, solver):
            lam_np = lame.detach().cpu().numpy().astype(np.float64)
            amp_np = amps.detach().cpu().numpy().astype(np.float64)
            if not (np.array_equal(lam_np, solver.lame) and np.array_equal(amp_np, solver.amps)):
                solver.set_parameters(lam_np, amp_np)
            u, _, _ = solver.solve(want_lambda=False)
            ctx.solver = solver
            ctx.params = (lam_np, amp_np)
            ctx.like = ((lame.device, lame.dtype), (amps.device, amps.dtype))
            ctx.save_for_backward(u)
            return u

        @staticmethod
        def backward(ctx, grad_u):
            (u,) = ctx.saved_tensors
            solver = ctx.solver
            lam_np, amp_np = ctx.params
            if not (np.array_equal(lam_np, solver.lame) and np.array_equal(amp_np, solver.amps)):
                solver.set_parameters(lam_np, amp_np)
            _, dlam, dmu, damp, _ = solver.solve_adjoint(grad_u.contiguous(), u)
            (ld, lt), (ad, at) = ctx.like
            g_lame = torch.from_numpy(np.stack([dlam, dmu], axis=1)).to(device=ld, dtype=lt)
            g_amps = torch.from_numpy(damp).to(device=ad, dtype=at)
            return g_lame, g_amps, None

    class _MassNorm(torch.autograd.Function):
        """0.5 e^T M e with the physical mass M of the handle."""

        @staticmethod
        def forward(ctx, e, solver):
            Me = solver.apply("mass", e.contiguous())
            ctx.save_for_backward(Me)
            return 0.5 * torch.dot(e, Me)

        @staticmethod
        def backward(ctx, g):
            (Me,) = ctx.saved_tensors
            return g * Me, None

    return _AfietiSolve, _MassNorm


def AfietiSolve(lame, amps, solver):
    """Differentiable AF-IETI solve: u(lame, amps) on ``solver``'s problems."""
    return _autograd()[0].apply(lame, amps, solver)


def mass_norm_loss(e, solver):
    """Differentiable 0.5 * e^T M e (physical mass of ``solver``)."""
    return _autograd()[1].apply(e, solver)
