"""Python binding: Operator handles, applies, solve and the autograd Function.

Argument marshalling only (tensor data pointers, the current stream); all
arithmetic runs in libtprec.so.
"""
import atexit
import ctypes as C
import weakref

import torch

from . import _lib as L


def _stream_ptr(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _prec(p):
    key = p.upper() if isinstance(p, str) else p
    if isinstance(key, str):
        if key not in L.PRECS:
            raise ValueError(f"precision {p!r}: one of {list(L.PRECS)}")
        return L.PRECS[key]
    return int(key)


def _torch_allocator(device):
    """tp_alloc_fn / tp_free_fn callbacks over torch's caching allocator on `device`."""
    # bound now: an operator released while the interpreter shuts down must not look up
    # module attributes that teardown may already have cleared
    alloc_fn, delete_fn = torch.cuda.caching_allocator_alloc, torch.cuda.caching_allocator_delete

    def alloc(nbytes, stream, user):
        try:
            return alloc_fn(int(nbytes), device=device, stream=int(stream or 0))
        except Exception:  # out of memory: the library reports TP_ENOMEM
            return None

    def free(ptr, nbytes, stream, user):
        delete_fn(int(ptr))

    return L.ALLOC_FN(alloc), L.FREE_FN(free)


# operators still open at exit are closed before torch's own exit handlers run
_open_ops = weakref.WeakSet()


@atexit.register
def _close_open_ops():
    for op in list(_open_ops):
        op.close()


def _scheme(s):
    if isinstance(s, str):
        if s.upper() not in L.SCHEMES:
            raise ValueError(f"scheme {s!r}: one of {list(L.SCHEMES)}")
        return L.SCHEMES[s.upper()]
    return int(s)


class Field:
    """A device buffer in one of the library's layouts (tp_field): `buf` holds nrhs right-hand
    sides back to back.  Internal layouts are opaque; an F64 FULL internal field read as a
    complex128 vector (as_complex) has the canonical field's inner products."""

    def __init__(self, buf, layout, prec, subset, nrhs):
        self.buf, self.layout, self.prec, self.subset, self.nrhs = buf, layout, prec, subset, nrhs

    def desc(self):
        return L.TpField(data=self.buf.data_ptr(), layout=L.LAYOUTS[self.layout], prec=L.PRECS[self.prec],
                         subset=L.SUBSETS[self.subset], nrhs=self.nrhs)

    def as_complex(self):
        if self.prec != "F64" or self.subset != "FULL" or self.layout == "CANONICAL":
            raise ValueError("as_complex: F64 FULL internal fields only")
        return self.buf.view(torch.complex128).view(self.nrhs, -1)


class Operator:
    """M = A + mu - D_t - D_s/gamma_f bound to a gauge field, on one GPU.

    links: complex128 tensor [4, Lt, Lz, Ly, Lx, 3, 3] (CPU or CUDA).
    c_s, c_t: the literal SW coefficients (both 0 for Wilson fermions).
    bc_t: +1 periodic or -1 antiperiodic in time.
    allocator: "torch" (default) hands every device allocation of the library to torch's
    caching allocator (tp_ctx_set_allocator); "hip" leaves it to hipMalloc.
    """

    def __init__(self, links, m0, gamma_f, c_s=0.0, c_t=0.0, bc_t=-1, device=0, allocator="torch"):
        self._lib = L.load()
        lib = self._lib
        if links.dtype != torch.complex128 or links.dim() != 7 or links.shape[0] != 4:
            raise ValueError("links must be complex128 [4, Lt, Lz, Ly, Lx, 3, 3]")
        lt, lz, ly, lx = links.shape[1:5]
        self.dims = (lx, ly, lz, lt)
        self.device = torch.device("cuda", device)
        self.m0, self.gamma_f, self.c_s, self.c_t, self.bc_t = m0, gamma_f, c_s, c_t, bc_t
        self._ctx = C.c_void_p()
        self._gauge = C.c_void_p()
        self._clover = C.c_void_p()
        self._op = C.c_void_p()
        d = (C.c_int32 * 4)(*self.dims)
        L.check(lib.tp_ctx_create(d, int(bc_t), int(device), C.byref(self._ctx)))
        self._bind_stream()
        self._alloc_cb = None
        _open_ops.add(self)
        if allocator == "torch":
            self._alloc_cb = _torch_allocator(device)
            L.check(lib.tp_ctx_set_allocator(self._ctx, self._alloc_cb[0], self._alloc_cb[1], None))
        elif allocator != "hip":
            raise ValueError(f"allocator {allocator!r}: 'torch' or 'hip'")
        links = links.contiguous()
        where = L.TP_DEVICE if links.is_cuda else L.TP_HOST
        L.check(lib.tp_gauge_create(self._ctx, C.c_void_p(links.data_ptr()), where,
                                    C.byref(self._gauge)))
        if c_s != 0.0 or c_t != 0.0:
            L.check(lib.tp_clover_create(self._gauge, float(c_s), float(c_t), C.byref(self._clover)))
        L.check(lib.tp_op_create(self._gauge, self._clover, float(m0), float(gamma_f),
                                 C.byref(self._op)))
        mu = C.c_double()
        L.check(lib.tp_op_mass(self._op, C.byref(mu)))
        self.mu = mu.value

    def set_cutoff(self, eps):
        """The cutoff trick of Sec. II.A (tp_op_set_cutoff): the Woodbury correction of the
        temporal inverses is dropped where its eq:cutoff bound is below eps (0: exact).
        Returns the number of time slices dropped at each line's suppressed end."""
        n = C.c_int32()
        L.check(self._lib.tp_op_set_cutoff(self._op, float(eps), C.byref(n)))
        return n.value

    def device_bytes(self):
        """Device memory held by the library for this operator (context and handles)."""
        n = C.c_size_t()
        L.check(self._lib.tp_ctx_device_bytes(self._ctx, C.byref(n)))
        return n.value

    # ---- plumbing --------------------------------------------------------------
    def _bind_stream(self):
        L.check(self._lib.tp_ctx_set_stream(self._ctx, _stream_ptr(self.device)))

    @property
    def spinor_shape(self):
        lx, ly, lz, lt = self.dims
        return (lt, lz, ly, lx, 4, 3)

    def _in(self, psi):
        if psi.dtype != torch.complex128 or tuple(psi.shape) != self.spinor_shape:
            raise ValueError(f"spinor must be complex128 {self.spinor_shape}")
        return psi.to(self.device).contiguous()

    def _out(self):
        return torch.empty(self.spinor_shape, dtype=torch.complex128, device=self.device)

    def _call(self, fn, *args):
        self._bind_stream()
        L.check(fn(*args))

    def close(self):
        lib = getattr(self, "_lib", None)
        if lib is None:
            return
        if self._op:
            lib.tp_op_destroy(self._op)
        if self._clover:
            lib.tp_clover_destroy(self._clover)
        if self._gauge:
            lib.tp_gauge_destroy(self._gauge)
        if self._ctx:
            lib.tp_ctx_destroy(self._ctx)
        self._op = self._clover = self._gauge = self._ctx = C.c_void_p()
        self._lib = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- applies -------------------------------------------------------------------
    def _unary(self, fn, psi, *extra):
        src = self._in(psi)
        dst = self._out()
        self._call(fn, self._op, *extra[:1], C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()),
                   *extra[1:])
        return dst

    def apply_M(self, psi, prec="F64", dagger=False):
        return self._unary(self._lib.tp_apply_M, psi, _prec(prec), int(dagger))

    def apply_Ds(self, psi, prec="F64"):
        return self._unary(self._lib.tp_apply_Ds, psi, _prec(prec))

    def apply_clover(self, psi, prec="F64", plus_mu=0):
        return self._unary(self._lib.tp_apply_clover, psi, _prec(prec), int(plus_mu))

    def apply_Tinv(self, psi, prec="F64", dagger=False):
        return self._unary(self._lib.tp_apply_Tinv, psi, _prec(prec), int(dagger))

    def apply_CL(self, psi, prec="F64"):
        return self._unary(self._lib.tp_apply_CL, psi, _prec(prec))

    def apply_CR(self, psi, prec="F64"):
        return self._unary(self._lib.tp_apply_CR, psi, _prec(prec))

    def apply_prec(self, psi, scheme, prec="F64", dagger=False):
        src = self._in(psi)
        dst = self._out()
        self._call(self._lib.tp_apply_prec, self._op, _scheme(scheme), _prec(prec),
                   C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), int(dagger))
        return dst

    def prepare_source(self, eta, scheme, prec="F64"):
        src = self._in(eta)
        dst = self._out()
        self._call(self._lib.tp_prepare_source, self._op, _scheme(scheme), _prec(prec),
                   C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()))
        return dst

    def reconstruct(self, y, scheme, prec="F64"):
        src = self._in(y)
        dst = self._out()
        self._call(self._lib.tp_reconstruct, self._op, _scheme(scheme), _prec(prec),
                   C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()))
        return dst

    # ---- fields in the library's layouts ------------------------------------------------
    def field_bytes(self, layout="P3", prec="F64", subset="FULL"):
        n = C.c_size_t()
        L.check(self._lib.tp_field_bytes(self._op, L.LAYOUTS[layout], _prec(prec), L.SUBSETS[subset],
                                         C.byref(n)))
        return n.value

    def field(self, layout="P3", prec="F64", subset="FULL", nrhs=1):
        """An uninitialised field (device memory from torch)."""
        if layout == "CANONICAL":
            t = torch.empty((nrhs,) + self.spinor_shape, dtype=torch.complex128, device=self.device)
            return Field(t, layout, "F64", "FULL", nrhs)
        per = self.field_bytes(layout, prec, subset)
        return Field(torch.empty(nrhs * per, dtype=torch.uint8, device=self.device), layout, prec, subset, nrhs)

    def _canonical(self, psi):
        psi = psi.to(self.device).contiguous()
        if psi.dtype != torch.complex128 or tuple(psi.shape[-6:]) != self.spinor_shape:
            raise ValueError(f"spinor must be complex128 {self.spinor_shape} (or a batch of them)")
        n = 1 if psi.dim() == 6 else psi.shape[0]
        return Field(psi.view((n,) + self.spinor_shape), "CANONICAL", "F64", "FULL", n)

    def convert_field(self, dst, src):
        self._call(self._lib.tp_field_convert, self._op, C.byref(dst.desc()), C.byref(src.desc()))
        return dst

    def to_field(self, psi, layout="P3", prec="F64", subset="FULL"):
        """A canonical spinor (or batch) converted into a field of the given layout."""
        src = self._canonical(psi)
        return self.convert_field(self.field(layout, prec, subset, src.nrhs), src)

    def from_field(self, f):
        """The canonical complex128 spinors [nrhs, Lt, Lz, Ly, Lx, 4, 3] of a field."""
        out = self.field("CANONICAL", nrhs=f.nrhs)
        self.convert_field(out, f)
        return out.buf

    def apply_prec_field(self, f, scheme, dagger=False, out=None):
        out = out if out is not None else self.field(f.layout, f.prec, f.subset, f.nrhs)
        self._call(self._lib.tp_apply_prec_field, self._op, _scheme(scheme), C.byref(out.desc()),
                   C.byref(f.desc()), int(dagger))
        return out

    def prepare_source_field(self, eta, scheme, prec="F64"):
        """eta~ = S_L eta as a FULL field of the scheme's layout; eta a canonical tensor or a field."""
        src = eta if isinstance(eta, Field) else self._canonical(eta)
        lay = "P4" if _scheme(scheme) == L.SCHEMES["SCHUR4D"] else "P3"
        out = self.field(lay, prec, "FULL", src.nrhs)
        self._call(self._lib.tp_prepare_source_field, self._op, _scheme(scheme), C.byref(out.desc()),
                   C.byref(src.desc()))
        return out

    def reconstruct_field(self, y, scheme):
        """x = S_R y as canonical spinors [nrhs, ...]."""
        out = self.field("CANONICAL", nrhs=y.nrhs)
        self._call(self._lib.tp_reconstruct_field, self._op, _scheme(scheme), C.byref(out.desc()),
                   C.byref(y.desc()))
        return out.buf

    # ---- solve -----------------------------------------------------------------------
    def solve(self, eta, scheme="TEMPORAL_SCHUR", solver="BICGSTAB", prec="F64", tol=1e-10,
              inner_tol=0.0, max_iter=0, max_restarts=0, x0=None, estimate_kappa=False,
              dagger=False, raise_on_noconv=True):
        """x with |eta - M x| <= tol |eta| (M^dagger with dagger); returns (x, info dict)."""
        src = self._in(eta)
        x = self._in(x0).clone() if x0 is not None else self._out()
        P = L.SolveParams(scheme=_scheme(scheme), solver=L.SOLVERS[solver.upper()], prec=_prec(prec),
                          max_iter=int(max_iter), max_restarts=int(max_restarts),
                          use_x0=int(x0 is not None), estimate_kappa=int(estimate_kappa),
                          dagger=int(bool(dagger)), tol=float(tol), inner_tol=float(inner_tol))
        info = L.SolveInfo()
        self._bind_stream()
        st = self._lib.tp_solve(self._op, C.byref(P), C.c_void_p(x.data_ptr()),
                                C.c_void_p(src.data_ptr()), C.byref(info))
        d = info.as_dict()
        d["status"] = st
        if st != L.TP_OK and (raise_on_noconv or st != L.TP_ENOCONV):
            L.check(st)
        return x, d

    def solve_multi(self, etas, scheme="TEMPORAL_SCHUR", solver="BICGSTAB", prec="F64", tol=1e-10,
                    inner_tol=0.0, max_iter=0, max_restarts=0, x0=None, dagger=False,
                    raise_on_noconv=True):
        """x[k] with |eta[k] - M x[k]| <= tol |eta[k]| for a batch of up to 16 sources solved
        together (tp_solve_multi); etas: [n, Lt, Lz, Ly, Lx, 4, 3].  Returns (x, [info])."""
        n = len(etas)
        srcs = [self._in(e) for e in etas]
        xs = [self._in(x0[k]).clone() if x0 is not None else self._out() for k in range(n)]
        P = L.SolveParams(scheme=_scheme(scheme), solver=L.SOLVERS[solver.upper()], prec=_prec(prec),
                          max_iter=int(max_iter), max_restarts=int(max_restarts),
                          use_x0=int(x0 is not None), estimate_kappa=0,
                          dagger=int(bool(dagger)), tol=float(tol), inner_tol=float(inner_tol))
        infos = (L.SolveInfo * n)()
        xp = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
        ep = (C.c_void_p * n)(*[e.data_ptr() for e in srcs])
        self._bind_stream()
        st = self._lib.tp_solve_multi(self._op, C.byref(P), n, xp, ep, infos)
        out = [infos[k].as_dict() for k in range(n)]
        for d in out:
            d["status"] = st
        if st != L.TP_OK and (raise_on_noconv or st != L.TP_ENOCONV):
            L.check(st)
        return torch.stack(xs), out

    def force(self, x, lam, projected=True, hopping_only=False):
        """Link gradient from x and lambda (see tp_force): [4, Lt, Lz, Ly, Lx, 3, 3]; with a
        clover term it includes the SW term's dependence on the links unless hopping_only."""
        xs, ls = self._in(x), self._in(lam)
        lx, ly, lz, lt = self.dims
        g = torch.empty((4, lt, lz, ly, lx, 3, 3), dtype=torch.complex128, device=self.device)
        self._call(self._lib.tp_force, self._op, C.c_void_p(xs.data_ptr()),
                   C.c_void_p(ls.data_ptr()), C.c_void_p(g.data_ptr()),
                   int(bool(projected)) | (2 if hopping_only else 0))
        return g

    def plaquette(self):
        ps, pt = C.c_double(), C.c_double()
        self._call(self._lib.tp_gauge_plaquette, self._gauge, C.byref(ps), C.byref(pt))
        return ps.value, pt.value

    # ---- per-kernel timing --------------------------------------------------------------
    def profile(self, on=True, only=None):
        """Per-kernel-group HIP-event timing; `only`: names of the groups to time (all if None)."""
        mask = 0xFFFFFFFF
        if only is not None:
            names = [self._lib.tp_prof_name(k).decode() for k in range(self._lib.tp_prof_count())]
            unknown = set(only) - set(names)
            if unknown:
                raise ValueError(f"unknown kernel groups {sorted(unknown)}; known: {names}")
            mask = sum(1 << names.index(n) for n in only)
        self._call(self._lib.tp_prof_select, self._ctx, mask)
        self._call(self._lib.tp_prof_enable, self._ctx, int(on))

    def profile_reset(self):
        self._call(self._lib.tp_prof_reset, self._ctx)

    def profile_stats(self):
        out = {}
        n = self._lib.tp_prof_count()
        for k in range(n):
            cnt, ms, by = C.c_int64(), C.c_double(), C.c_double()
            self._call(self._lib.tp_prof_get, self._ctx, k, C.byref(cnt), C.byref(ms), C.byref(by))
            if cnt.value:
                out[self._lib.tp_prof_name(k).decode()] = dict(launches=cnt.value, ms=ms.value,
                                                                bytes=by.value)
        return out


def solve(links, eta, m0, gamma_f, c_s=0.0, c_t=0.0, bc_t=-1, **kw):
    op = Operator(links, m0, gamma_f, c_s, c_t, bc_t)
    try:
        return op.solve(eta, **kw)
    finally:
        op.close()


class SolveFn(torch.autograd.Function):
    """x = M(U)^-1 eta with a hand-written backward.

    Backward: lambda solves M^dagger lambda = g (tp_solve with dagger, the same
    preconditioned solver), grad_eta = lambda, and grad_U is the link gradient
    (tp_force, raw form), including the SW term's dependence on the links.
    Conventions follow torch: dL = Re <grad, dz>.
    """

    @staticmethod
    def forward(ctx, links, eta, m0, gamma_f, c_s=0.0, c_t=0.0, bc_t=-1, scheme="TEMPORAL_SCHUR",
                prec="F64", tol=1e-10):
        op = Operator(links.detach(), m0, gamma_f, c_s, c_t, bc_t, device=eta.device.index or 0)
        x, _ = op.solve(eta.detach(), scheme=scheme, prec=prec, tol=tol)
        ctx.op = op
        ctx.opts = dict(scheme=scheme, prec=prec, tol=tol)
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        op = ctx.op
        lam, _ = op.solve(g.contiguous(), dagger=True, **ctx.opts)
        grad_links = op.force(x, lam, projected=False) if ctx.needs_input_grad[0] else None
        op.close()
        ctx.op = None
        return grad_links, lam, None, None, None, None, None, None, None, None
