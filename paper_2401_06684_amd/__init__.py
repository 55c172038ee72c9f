"""MI355X-native polynomially preconditioned Krylov approximation of A^{-1/2} b
and A^{1/2} b (Frommer, Ramirez-Hidalgo, Schweitzer, Tsolakis, arXiv 2401.06684).

Thin binding over the C ABI of ``libfa.so`` (include/fa.h): every step of the
method runs in the library's HIP kernels and host runtime; this module only
marshals arguments.  PyTorch provides device memory and the current stream.

    import torch, paper_2401_06684_amd as fa
    op = fa.Stencil7((nx, ny, nz), coeffs)          # or fa.CSR(...), fa.Wilson(...)
    op.poly_setup(16)                                # Chebyshev on the exact interval
    x, stats = op.apply(b, kind="invsqrt", m_max=200, tol=1e-8)
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from ._lib import (FA_C128, FA_F64, FA_FORCE_ARNOLDI, FA_HERMITIAN, FA_INVSQRT,  # noqa: F401
                   FA_MIXED, FA_NO_FUSION, FA_POLY_AUTO, FA_POLY_CHEB, FA_POLY_HARMONIC,
                   FA_POLY_LS, FA_POLY_RITZ, FA_PROFILE, FA_Q2, FA_RIGHT_PREC, FA_SQRT,
                   FA_TWO_PASS, FAError, check, lib)

__all__ = ["Stencil7", "CSR", "Wilson", "Server", "FAError", "lib", "dense_invsqrt_e1",
           "dense_tridiag_invsqrt_e1"]

_KIND = {"invsqrt": FA_INVSQRT, "sqrt": FA_SQRT}
_METHOD = {"auto": FA_POLY_AUTO, "cheb": FA_POLY_CHEB, "ritz": FA_POLY_RITZ,
           "harmonic": FA_POLY_HARMONIC, "ls": FA_POLY_LS}


def _fuse_flags(fuse):
    """Flags for the most recurrence terms per launch: True or 4, 3, 2, False or 1."""
    if fuse is True or fuse == 4:
        return 0
    if fuse is False or fuse == 1:
        return FA_NO_FUSION
    if fuse == 2:
        return _lib.FA_FUSE2
    if fuse == 3:
        return _lib.FA_FUSE3
    raise ValueError("fuse must be True, False, 1, 2, 3 or 4")


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def workspace(nbytes, device):
    """A 256-byte aligned device buffer of nbytes (torch-owned)."""
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, C.c_void_p(buf.data_ptr() + off), int(nbytes)


class Operator:
    """Common part of all operators: polynomial setup and fa_apply."""

    dtype = torch.float64

    def __init__(self, handle, device, keep):
        self._h = handle
        self.device = device
        self._keep = keep  # borrowed device arrays stay alive with the op
        n = C.c_int64()
        dt = C.c_int()
        check(lib().fa_op_info(self._h, C.byref(n), C.byref(dt)), "fa_op_info")
        self.n = n.value
        self.dtype = torch.complex128 if dt.value == FA_C128 else torch.float64
        self._ws = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                lib().fa_destroy(h)
            except Exception:
                pass
            self._h = None

    # ---- spectral interval / polynomial ----------------------------------
    def set_spectral_interval(self, lo, hi):
        check(lib().fa_set_spectral_interval(self._h, lo, hi), "fa_set_spectral_interval")

    def spectral_interval(self):
        lo, hi = C.c_double(), C.c_double()
        st = lib().fa_get_spectral_interval(self._h, C.byref(lo), C.byref(hi))
        if st == _lib.FA_ERR_NO_INTERVAL:
            return None
        check(st, "fa_get_spectral_interval")
        return lo.value, hi.value

    def poly_setup(self, degree, method="auto", start=None, ritz_steps=60, r_min=0.1,
                   step=0.005):
        """Choose q of the given degree (0: plain method).
        method: auto|cheb|ritz|harmonic|ls.

        For (harmonic) Ritz and least-squares polynomials `start` is the start
        vector of the setup Arnoldi run (a device tensor of length n); ls uses
        ritz_steps Arnoldi steps and the contour parameters r_min and step.
        """
        m = _METHOD[method]
        if m == FA_POLY_LS:
            nbytes = lib().fa_poly_workspace_bytes(self._h, ritz_steps - 1, FA_POLY_RITZ)
        else:
            nbytes = lib().fa_poly_workspace_bytes(self._h, degree, m)
        keep = None
        wsp = C.c_void_p(0)
        if nbytes:
            keep, wsp, nbytes = workspace(nbytes, self.device)
        sp = C.c_void_p(0)
        if start is not None:
            start = self._vec(start, "start")
            sp = _ptr(start)
        if m == FA_POLY_LS and degree > 0:
            st = lib().fa_poly_setup_ls(self._h, degree, ritz_steps, float(r_min), float(step),
                                        sp, wsp, nbytes, _stream(self.device))
        else:
            st = lib().fa_poly_setup(self._h, degree, m, sp, wsp, nbytes, _stream(self.device))
        check(st, "fa_poly_setup")
        del keep

    def poly(self):
        """The polynomial as a dict (method, degree, coefficients, nodes, ...)."""
        deg, meth = C.c_int(), C.c_int()
        check(lib().fa_poly_get(self._h, C.byref(deg), C.byref(meth), None, None, None, None,
                                None, None), "fa_poly_get")
        K = deg.value
        arr = lambda: (C.c_double * (K + 1))()  # noqa: E731
        cr, ci, nr, ni = arr(), arr(), arr(), arr()
        iv = (C.c_double * 2)()
        rho = C.c_double()
        check(lib().fa_poly_get(self._h, None, None, cr, ci, nr, ni, iv, C.byref(rho)),
              "fa_poly_get")
        meth_name = {-1: "one", FA_POLY_CHEB: "cheb", FA_POLY_RITZ: "ritz",
                     FA_POLY_HARMONIC: "harmonic", FA_POLY_LS: "ls"}[meth.value]
        out = {"method": meth_name, "degree": K}
        if meth_name == "cheb":
            out.update(c=list(cr), interval=(iv[0], iv[1]))
        elif meth_name in ("ritz", "harmonic"):
            out.update(eta=[complex(a, b) for a, b in zip(cr, ci)],
                       theta=[complex(a, b) for a, b in zip(nr, ni)], rho=rho.value)
        elif meth_name == "ls":
            npts = C.c_int64()
            hr, hi = (C.c_double * ((K + 1) * K))(), (C.c_double * ((K + 1) * K))()
            check(lib().fa_poly_get_ls(self._h, C.byref(npts), hr, hi), "fa_poly_get_ls")
            h = [[complex(hr[j * (K + 1) + i], hi[j * (K + 1) + i]) for j in range(K)]
                 for i in range(K + 1)]
            out.update(alpha=[complex(a, b) for a, b in zip(cr, ci)], npts=npts.value, h=h)
        return out

    # ---- application -------------------------------------------------------
    def _vec(self, v, name):
        if not (isinstance(v, torch.Tensor) and v.is_cuda):
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if v.dtype != self.dtype or v.numel() != self.n or not v.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {self.dtype} tensor of {self.n} entries")
        return v

    def workspace_bytes(self, m_max, flags=0):
        return lib().fa_workspace_bytes(self._h, m_max, flags)

    def _workspace(self, m_max, flags=0):
        # one cached workspace per stream: calls on different streams may
        # overlap, and a workspace must not be shared by overlapping calls
        nbytes = self.workspace_bytes(m_max, flags)
        key = ("apply", torch.cuda.current_stream(self.device).cuda_stream)
        ws = self._ws.get(key)
        if ws is None or ws[2] < nbytes:
            self._ws.pop(key, None)
            ws = workspace(nbytes, self.device)
            self._ws[key] = ws
        return ws

    def release_workspace(self):
        self._ws.clear()

    def apply(self, b, kind="invsqrt", m_max=100, tol=1e-10, check_every=0, out=None,
              force_arnoldi=False, profile=False, fuse=True, mixed=False, two_pass=False,
              right=False, orth="dcgs2", raise_not_converged=False):
        """x ~ A^{-1/2} b or A^{1/2} b.  Returns (x, stats dict).

        fuse: most recurrence terms per launch on a 7-point stencil (True = 4,
        3, 2, or False / 1 for one launch per term);
        mixed=True runs the polynomial chain in FP32 (stencil, Chebyshev q);
        two_pass=True runs two-pass Lanczos (O(n) basis storage);
        right=True runs the right-preconditioned variant (Algorithm 2; with
        two_pass only at a fixed m, tol <= 0);
        orth="cgs2" runs both Gram-Schmidt passes in every Arnoldi step
        (default "dcgs2": the second pass delayed by one step).
        """
        if orth not in ("dcgs2", "cgs2"):
            raise ValueError("orth must be 'dcgs2' or 'cgs2'")
        b = self._vec(b, "b")
        x = out if out is not None else torch.empty_like(b)
        self._vec(x, "out")
        flags = ((FA_FORCE_ARNOLDI if force_arnoldi else 0) | (FA_PROFILE if profile else 0)
                 | _fuse_flags(fuse) | (FA_MIXED if mixed else 0)
                 | (FA_TWO_PASS if two_pass else 0) | (FA_RIGHT_PREC if right else 0)
                 | (_lib.FA_CGS2 if orth == "cgs2" else 0))
        _, wsp, nbytes = self._workspace(m_max, flags)
        stats = _lib.fa_stats()
        st = lib().fa_apply(self._h, _KIND[kind], _ptr(b), _ptr(x), m_max, float(tol),
                            check_every, wsp, nbytes, flags, _stream(self.device),
                            C.byref(stats))
        check(st, "fa_apply")
        if st == _lib.FA_WARN_NOT_CONVERGED and raise_not_converged:
            raise FAError(st, "fa_apply")
        d = stats.as_dict()
        d["status"] = st
        return x, d

    def apply_noalloc(self, b, kind="invsqrt", m_max=100, tol=1e-10, check_every=0, out=None,
                      fuse=True, mixed=False, orth="dcgs2"):
        """apply() through fa_apply_noalloc: the solve runs in the library's
        static device array (FA_NOALLOC_MAX_BYTES), no workspace is passed.
        Returns (x, stats dict)."""
        if orth not in ("dcgs2", "cgs2"):
            raise ValueError("orth must be 'dcgs2' or 'cgs2'")
        b = self._vec(b, "b")
        x = out if out is not None else torch.empty_like(b)
        self._vec(x, "out")
        flags = _fuse_flags(fuse) | (FA_MIXED if mixed else 0) | (
            _lib.FA_CGS2 if orth == "cgs2" else 0)
        stats = _lib.fa_stats()
        st = lib().fa_apply_noalloc(self._h, _KIND[kind], _ptr(b), _ptr(x), m_max, float(tol),
                                    check_every, flags, _stream(self.device), C.byref(stats))
        check(st, "fa_apply_noalloc")
        d = stats.as_dict()
        d["status"] = st
        return x, d

    def block_apply(self, B, kind="invsqrt", m_max=30, tol=1e-10, check_every=0, out=None,
                    mixed=False, graph=False, raise_not_converged=False):
        """X ~ A^{-1/2} B or A^{1/2} B for the columns of B (n x s, s in
        {16, 32, 64}, a contiguous row-major tensor) by block Arnoldi.
        graph=True replays the block steps from captured HIP graphs.
        Returns (X, stats dict)."""
        if not (isinstance(B, torch.Tensor) and B.is_cuda and B.dtype == torch.float64
                and B.dim() == 2 and B.shape[0] == self.n and B.is_contiguous()):
            raise ValueError(f"B must be a contiguous float64 CUDA tensor of shape ({self.n}, s)")
        s = B.shape[1]
        X = out if out is not None else torch.empty_like(B)
        if X.shape != B.shape or not X.is_contiguous() or X.dtype != B.dtype:
            raise ValueError("out must match B")
        flags = (FA_MIXED if mixed else 0) | (_lib.FA_GRAPH if graph else 0)
        nbytes = lib().fa_block_workspace_bytes(self._h, s, m_max, flags)
        if nbytes == 0:
            raise ValueError("unsupported block size (s must be 16, 32 or 64)")
        ws = self._ws.get("block")
        if ws is None or ws[2] < nbytes:
            self._ws.pop("block", None)
            ws = workspace(nbytes, self.device)
            self._ws["block"] = ws
        stats = _lib.fa_block_stats()
        cur = torch.cuda.current_stream(self.device)
        run = cur
        if graph and cur.cuda_stream == 0:
            # graphs are captured on the stream given; the null stream cannot be
            run = self._ws.get("graph_stream")
            if run is None:
                run = self._ws["graph_stream"] = torch.cuda.Stream(self.device)
            run.wait_stream(cur)
        st = lib().fa_block_apply(self._h, _KIND[kind], s, _ptr(B), _ptr(X), int(m_max),
                                  float(tol), int(check_every), ws[1], ws[2], flags,
                                  C.c_void_p(run.cuda_stream), C.byref(stats))
        if run is not cur:
            cur.wait_stream(run)
        check(st, "fa_block_apply")
        if st == _lib.FA_WARN_NOT_CONVERGED and raise_not_converged:
            raise FAError(st, "fa_block_apply")
        d = stats.as_dict()
        d["status"] = st
        return X, d

    def op_apply(self, x, out=None, split_long_rows=True):
        """y = A x (one operator application).  A CSR op splits rows of more
        than 4096 entries over several workgroups in a scratch workspace
        (split_long_rows=False: one workgroup per such row, the same bits);
        a squared Wilson op always takes the workspace (for Q x)."""
        x = self._vec(x, "x")
        y = out if out is not None else torch.empty_like(x)
        wsp, nbytes = C.c_void_p(0), 0
        if split_long_rows or getattr(self, "squared", False):
            _, wsp, nbytes = self._workspace(1)
        check(lib().fa_op_apply(self._h, _ptr(x), _ptr(y), wsp, nbytes, _stream(self.device)),
              "fa_op_apply")
        return y

    def poly_apply(self, x, out=None):
        """y = q(A) x."""
        x = self._vec(x, "x")
        y = out if out is not None else torch.empty_like(x)
        nbytes = lib().fa_workspace_bytes(self._h, 1, 0)
        keep, wsp, nbytes = workspace(nbytes, self.device)
        check(lib().fa_poly_apply(self._h, _ptr(x), _ptr(y), wsp, nbytes, _stream(self.device)),
              "fa_poly_apply")
        torch.cuda.current_stream(self.device).synchronize()
        del keep
        return y


class Stencil7(Operator):
    """Real 7-point (nz > 1) or 5-point (nz = 1) stencil, zero Dirichlet boundary.

    coeffs = [c0, c_xm, c_xp, c_ym, c_yp, c_zm, c_zp]; vectors are x-fastest.
    """

    def __init__(self, dims, coeffs, hermitian=False, device="cuda"):
        nx, ny, nz = (int(d) for d in dims)
        h = C.c_void_p()
        d4 = (C.c_int32 * 4)(nx, ny, nz, 1)
        c7 = (C.c_double * 7)(*[float(c) for c in coeffs])
        st = lib().fa_create_stencil(C.byref(h), _lib.FA_STENCIL7, d4, c7, 7, None,
                                     FA_HERMITIAN if hermitian else 0, None, 0, None)
        check(st, "fa_create_stencil")
        super().__init__(h, torch.device(device), None)
        self.dims = (nx, ny, nz)


class CSR(Operator):
    """Sparse matrix in CSR form (int32 indices; float64 or complex128 values)."""

    def __init__(self, rowptr, colind, vals, hermitian=False, device="cuda"):
        dev = torch.device(device)
        rp = torch.as_tensor(rowptr).to(device=dev, dtype=torch.int32).contiguous()
        ci = torch.as_tensor(colind).to(device=dev, dtype=torch.int32).contiguous()
        va = torch.as_tensor(vals).to(device=dev).contiguous()
        if va.dtype not in (torch.float64, torch.complex128):
            va = va.to(torch.float64)
        dt = FA_C128 if va.dtype == torch.complex128 else FA_F64
        n = rp.numel() - 1
        # operator memory (the library's list of long rows), owned by torch
        mem, mp, mb = workspace(lib().fa_op_device_bytes(_lib.FA_CSR, None, n, ci.numel()), dev)
        h = C.c_void_p()
        st = lib().fa_create_csr(C.byref(h), n, ci.numel(), _ptr(rp), _ptr(ci), _ptr(va), dt,
                                 FA_HERMITIAN if hermitian else 0, mp, mb, _stream(dev))
        check(st, "fa_create_csr")
        super().__init__(h, dev, (rp, ci, va, mem))


class Wilson(Operator):
    """Wilson-Dirac-like operator on a periodic 4D lattice (12 complex per site).

    links: complex128 tensor [4][Lt][Lz][Ly][Lx][3][3] (mu = x, y, z, t).
    mu: chemical potential on the temporal hops.  squared=True makes the op
    A = Q^2 with Q = Gamma_5 D (Sec. 6, Example 2: sign(Q) b = Q (Q^2)^{-1/2} b);
    hermitian=True (only with squared and mu = 0) selects Lanczos.
    """

    def __init__(self, links, m0, device="cuda", mu=0.0, squared=False, hermitian=False):
        dev = torch.device(device)
        U = torch.as_tensor(links).to(device=dev, dtype=torch.complex128).contiguous()
        if U.dim() != 7 or U.shape[0] != 4 or tuple(U.shape[-2:]) != (3, 3):
            raise ValueError("links must have shape (4, Lt, Lz, Ly, Lx, 3, 3)")
        Lt, Lz, Ly, Lx = (int(s) for s in U.shape[1:5])
        h = C.c_void_p()
        d4 = (C.c_int32 * 4)(Lx, Ly, Lz, Lt)
        p = (C.c_double * 2)(float(m0), float(mu))
        flags = (FA_Q2 if squared else 0) | (FA_HERMITIAN if hermitian else 0)
        # operator memory for the library's reordered copy of the links
        mem, mp, mb = workspace(lib().fa_op_device_bytes(_lib.FA_WILSON4D, d4, 0, 0), dev)
        # the library copies the links (reordered) on this stream and waits
        st = lib().fa_create_stencil(C.byref(h), _lib.FA_WILSON4D, d4, p, 2, _ptr(U), flags,
                                     mp, mb, _stream(dev))
        check(st, "fa_create_stencil")
        super().__init__(h, dev, (mem,))
        self.lattice = (Lt, Lz, Ly, Lx)
        self.squared = bool(squared)


class Server:
    """Request loop of f(A)b solves with admission by workspace memory.

    pool_bytes of device memory are carved into per-request workspaces (the
    Krylov basis and scratch); up to n_workers solves run at once, each on its
    own HIP stream.  submit() returns a ticket at once; wait(ticket) returns
    (x, info) when the solve is done.
    """

    def __init__(self, pool_bytes, n_workers=4, device="cuda"):
        self.device = torch.device(device)
        self._pool, pp, nbytes = workspace(pool_bytes, self.device)
        # one torch stream (default priority) per worker
        self._streams = [torch.cuda.Stream(self.device) for _ in range(int(n_workers))]
        sp = (C.c_void_p * len(self._streams))(*[s.cuda_stream for s in self._streams])
        torch.cuda.synchronize(self.device)
        h = C.c_void_p()
        check(lib().fa_server_create(C.byref(h), pp, nbytes, int(n_workers), sp),
              "fa_server_create")
        self._h = h
        self._live = {}

    def submit(self, op, b, kind="invsqrt", m_max=100, tol=1e-10, check_every=0, out=None,
               force_arnoldi=False, fuse=True, mixed=False, two_pass=False, right=False):
        """Queue one solve; b (and out) must stay untouched until it is done."""
        b = op._vec(b, "b")
        x = out if out is not None else torch.empty_like(b)
        op._vec(x, "out")
        flags = ((FA_FORCE_ARNOLDI if force_arnoldi else 0) | _fuse_flags(fuse)
                 | (FA_MIXED if mixed else 0) | (FA_TWO_PASS if two_pass else 0)
                 | (FA_RIGHT_PREC if right else 0))
        # b is produced on torch's stream; the server's streams do not wait for it
        torch.cuda.current_stream(self.device).synchronize()
        t = C.c_uint64()
        check(lib().fa_server_submit(self._h, op._h, _KIND[kind], _ptr(b), _ptr(x), int(m_max),
                                     float(tol), int(check_every), flags, C.byref(t)),
              "fa_server_submit")
        self._live[t.value] = (op, b, x)
        return t.value

    def poll(self, ticket):
        d = C.c_int()
        check(lib().fa_server_poll(self._h, ticket, C.byref(d)), "fa_server_poll")
        return bool(d.value)

    def wait(self, ticket, raise_errors=True):
        """Block until the solve is done; returns (x, info dict)."""
        info = _lib.fa_request_info()
        st = lib().fa_server_wait(self._h, ticket, C.byref(info))
        op, b, x = self._live.pop(ticket)
        if raise_errors:
            check(st, "fa_server_wait")
        d = {"status": info.status, "worker": info.worker, "stats": info.stats.as_dict(),
             "t_submit_ms": info.t_submit_ms, "t_start_ms": info.t_start_ms,
             "t_done_ms": info.t_done_ms, "ws_bytes": info.ws_bytes}
        return x, d

    def status(self):
        si = _lib.fa_server_info()
        check(lib().fa_server_status(self._h, C.byref(si)), "fa_server_status")
        return si.as_dict()

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib().fa_server_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dense_invsqrt_e1(H, beta):
    """Host routine: H^{-1/2} (beta e_1) for an upper Hessenberg numpy array."""
    import numpy as np
    H = np.asarray(H)
    m = H.shape[0]
    cplx = np.iscomplexobj(H)
    flat = np.ascontiguousarray(H.astype(np.complex128 if cplx else np.float64).reshape(-1, order="F"))
    src = flat.view(np.float64) if cplx else flat
    z = np.zeros(2 * m if cplx else m)
    dp = C.POINTER(C.c_double)
    st = lib().fa_dense_invsqrt_e1(m, FA_C128 if cplx else FA_F64, src.ctypes.data_as(dp), m,
                                   float(beta), z.ctypes.data_as(dp))
    check(st, "fa_dense_invsqrt_e1")
    return z.view(np.complex128) if cplx else z


def dense_tridiag_invsqrt_e1(alpha, offd, beta):
    """Host routine: T^{-1/2} (beta e_1) for a symmetric tridiagonal T."""
    import numpy as np
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    o = np.ascontiguousarray(offd, dtype=np.float64)
    if o.size == 0:
        o = np.zeros(1)
    z = np.zeros(a.size)
    dp = C.POINTER(C.c_double)
    st = lib().fa_dense_tridiag_invsqrt_e1(a.size, a.ctypes.data_as(dp), o.ctypes.data_as(dp),
                                           float(beta), z.ctypes.data_as(dp))
    check(st, "fa_dense_tridiag_invsqrt_e1")
    return z
