"""Python face of the C ABI: marshals numpy meshes and torch tensors."""
import ctypes as C
import json

import numpy as np

from . import _lib
from ._lib import CmError, check, lib


def _precond_code(precond):
    """False/None -> 0, True/"sai" -> 1 (the SAI), "cmp" -> 2 (Calderon)."""
    if isinstance(precond, str):
        if precond not in ("sai", "cmp"):
            raise ValueError("precond must be a bool, 'sai' or 'cmp'")
        return 1 if precond == "sai" else 2
    return 1 if precond else 0


class Operator:
    """MLFMA operator of one mesh at one wavenumber.

    Parameters mirror ``cm_opts``: nlv (levels including level 0), d0 (digits
    of the truncation rule, eq. (30)), interp_p (local Lagrange points),
    max_cols (largest batch).  host_only=True builds only the host plan (no
    GPU needed); deriv=True also builds dZ/dk tables; wide_near=True selects
    the two-box buffer at the two finest levels (CM_FLAG_WIDE_NEAR);
    autotune=True times the matrix-core interpolation variants per level at
    create and keeps the fastest (CM_FLAG_AUTOTUNE); r_standard=True gives
    R x the standard MLFMA lists instead of the sibling bookkeeping
    (CM_FLAG_R_STANDARD); k_sampling: the wavenumber at which the
    truncation rule sets L and the sampling (None: k itself; a common value
    freezes the discretisation across handles at nearby k); verbose=True
    makes the eigen-solvers print a progress line per restart to stderr;
    m2l_tile16=True selects the 16-box-tile FP32 translation kernel
    (CM_FLAG_M2L_TILE16) instead of the 64-box shared-source one;
    m2l_single_tiles=True makes single-column translations use the 16-box
    receiver tiles instead of the receiver-major kernel
    (CM_FLAG_M2L_SINGLE_TILES; same bits).  k may be a
    sequence of wavenumbers (a sweep; apply's k_index picks one per column);
    sweep_shared=True gives all of them the sampling of the largest (or of
    k_sampling) and runs FP32 Z / Z^H batches that span several wavenumbers
    as one pass (CM_FLAG_SWEEP_SHARED).
    """

    def __init__(self, V, F, k, nlv, d0=3.0, interp_p=6, eta=None, max_cols=32, host_only=False,
                 deriv=False, check_coverage=False, matrix_cores=True, near_fp32=False, wide_near=False,
                 autotune=False, r_standard=False, k_sampling=None, verbose=False, m2l_tile16=False,
                 m2l_single_tiles=False, sweep_shared=False, stream=None):
        L = lib()
        V = np.ascontiguousarray(V, dtype=np.float64)
        F = np.ascontiguousarray(F, dtype=np.int32)
        o = _lib.cm_opts()
        L.cm_default_opts(C.byref(o))
        o.nlv = int(nlv)
        o.d0 = float(d0)
        o.interp_p = int(interp_p)
        if eta is not None:
            o.eta = float(eta)
        o.max_cols = int(max_cols)
        o.k_sampling = float(k_sampling) if k_sampling else 0.0
        o.flags = ((_lib.CM_FLAG_HOST_ONLY if host_only else 0) | (_lib.CM_FLAG_DERIV if deriv else 0)
                   | (_lib.CM_FLAG_CHECK if check_coverage else 0)
                   | (0 if matrix_cores else _lib.CM_FLAG_NO_MATRIX_CORES)
                   | (_lib.CM_FLAG_NEAR_FP32 if near_fp32 else 0)
                   | (_lib.CM_FLAG_WIDE_NEAR if wide_near else 0)
                   | (_lib.CM_FLAG_AUTOTUNE if autotune else 0)
                   | (_lib.CM_FLAG_R_STANDARD if r_standard else 0)
                   | (_lib.CM_FLAG_VERBOSE if verbose else 0)
                   | (_lib.CM_FLAG_M2L_TILE16 if m2l_tile16 else 0)
                   | (_lib.CM_FLAG_M2L_SINGLE_TILES if m2l_single_tiles else 0)
                   | (_lib.CM_FLAG_SWEEP_SHARED if sweep_shared else 0))
        kk = np.atleast_1d(np.asarray(k, dtype=np.float64)).copy()
        h = C.c_void_p()
        s = self._stream_ptr(stream) if not host_only else None
        st = L.cm_create(V.ctypes.data, V.shape[0], F.ctypes.data, F.shape[0], kk.ctypes.data, len(kk), C.byref(o), s,
                         C.byref(h))
        check(st)
        self._h = h
        self._dev_index = None
        if not host_only:
            import torch
            self._dev_index = torch.cuda.current_device()   # the device the handle's tables live on
        self.ks = [float(v) for v in kk]   # the sweep's wavenumbers (k_index selects one per column)
        self.k = self.ks[0]
        self.host_only = host_only
        self.max_cols = int(max_cols)
        n = C.c_int64()
        check(L.cm_num_unknowns(h, C.byref(n)))
        self.N = int(n.value)

    @staticmethod
    def _stream_ptr(stream):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        return C.c_void_p(stream.cuda_stream)

    def close(self):
        if getattr(self, "_h", None):
            lib().cm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ host queries
    def rwg_table(self):
        e = np.zeros((self.N, 2), dtype=np.int32)
        t = np.zeros((self.N, 2), dtype=np.int32)
        check(lib().cm_rwg_table(self._h, e.ctypes.data, t.ctypes.data))
        return e, t

    def stats(self):
        need = C.c_int64()
        lib().cm_stats(self._h, None, 0, C.byref(need))
        buf = C.create_string_buffer(int(need.value))
        check(lib().cm_stats(self._h, buf, need.value, C.byref(need)))
        return json.loads(buf.value.decode())

    def stage_timing(self, enable=True):
        """Enable (or disable) HIP-event timing of every kernel stage."""
        check(lib().cm_stage_timing(self._h, 1 if enable else 0))

    def stage_times(self):
        """{stage: {"ms": total milliseconds, "calls": launches}} since stage_timing()."""
        need = C.c_int64()
        lib().cm_stage_times(self._h, None, 0, C.byref(need))
        buf = C.create_string_buffer(int(need.value) + 256)
        check(lib().cm_stage_times(self._h, buf, need.value + 256, C.byref(need)))
        return json.loads(buf.value.decode())

    def export_near(self, which=0):
        """Near-field (which=0), dZ_near/dk (1) or SAI (2) matrix as scipy CSR
        in public unknown order."""
        import scipy.sparse as sp
        nnz = C.c_int64()
        check(lib().cm_export_near(self._h, which, C.byref(nnz), None, None, None))
        ptr = np.zeros(self.N + 1, dtype=np.int64)
        col = np.zeros(nnz.value, dtype=np.int32)
        val = np.zeros(2 * nnz.value, dtype=np.float64)
        check(lib().cm_export_near(self._h, which, C.byref(nnz), ptr.ctypes.data, col.ctypes.data,
                                   val.ctypes.data))
        return sp.csr_matrix((val[0::2] + 1j * val[1::2], col, ptr), shape=(self.N, self.N))

    # ------------------------------------------------------------ device applies
    def _device(self):
        import torch
        return torch.device("cuda", torch.cuda.current_device())

    def _check_device(self, t):
        if self._dev_index is not None and t.device.index != self._dev_index:
            raise ValueError(f"tensor on {t.device}, operator built on cuda:{self._dev_index}")

    def _vec_args(self, x, out):
        """x as a row-major (N, ncols) view with unit column stride, and an
        output of the same dtype, shape, device and row stride."""
        import torch
        if not isinstance(x, torch.Tensor) or not x.is_cuda:
            raise TypeError("x must be a CUDA (HIP) torch tensor")
        if x.dtype not in (torch.complex64, torch.complex128):
            raise TypeError("x must be complex64 or complex128")
        squeeze = x.dim() == 1
        X = x.reshape(-1, 1) if squeeze else x
        if X.dim() != 2:
            raise ValueError("x must have shape (N,) or (N, ncols)")
        if X.shape[0] != self.N:
            raise ValueError(f"x has {X.shape[0]} rows, operator has N={self.N}")
        self._check_device(X)
        if X.stride(1) != 1 or X.stride(0) < X.shape[1]:
            X = X.contiguous()
        if out is None:
            # same row stride as X (a column slice of a wider tensor keeps its stride)
            out = torch.empty_strided(X.shape, (X.stride(0), 1), dtype=X.dtype, device=X.device)
        else:
            if not isinstance(out, torch.Tensor) or not out.is_cuda:
                raise TypeError("out must be a CUDA (HIP) torch tensor")
            if out.dim() == 1:
                out = out.reshape(-1, 1)
            if out.dtype != X.dtype:
                raise TypeError(f"out has dtype {out.dtype}, x has {X.dtype}")
            if tuple(out.shape) != tuple(X.shape):
                raise ValueError(f"out has shape {tuple(out.shape)}, x has {tuple(X.shape)}")
            if out.device != X.device:
                raise ValueError("out and x are on different devices")
            if out.stride(1) != 1 or out.stride(0) != X.stride(0):
                raise ValueError("out must be row-major with the same row stride as x")
        dt = _lib.CM_C128 if X.dtype == torch.complex128 else _lib.CM_C64
        return X, out, dt, squeeze

    def _start_vector(self, v0):
        """v0 checked for the Krylov drivers: complex128, N entries, CUDA."""
        import torch
        if not isinstance(v0, torch.Tensor) or not v0.is_cuda:
            raise TypeError("v0 must be a CUDA (HIP) torch tensor")
        if v0.dtype != torch.complex128:
            raise TypeError("v0 must be complex128")
        if v0.numel() != self.N:
            raise ValueError(f"v0 has {v0.numel()} entries, operator has N={self.N}")
        self._check_device(v0)
        return v0.reshape(-1).contiguous()

    @staticmethod
    def _k_index(k_index, ncols):
        if k_index is None:
            return None
        ki = np.ascontiguousarray(np.asarray(k_index, dtype=np.int32).reshape(-1))
        if ki.size != ncols:
            raise ValueError("k_index needs one entry per column")
        return ki

    def apply(self, x, op="Z", out=None, stream=None, k_index=None):
        """y = op(x) for x of shape (N,) or (N, ncols) on the GPU; k_index: one
        index into the handle's wavenumbers per column (None: all at k[0])."""
        X, Y, dt, squeeze = self._vec_args(x, out)
        ki = self._k_index(k_index, X.shape[1])
        st = lib().cm_apply(self._h, _lib.OPS[op], C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()),
                            X.stride(0), X.shape[1], None if ki is None else C.c_void_p(ki.ctypes.data),
                            dt, self._stream_ptr(stream))
        check(st)
        return Y.reshape(-1) if squeeze else Y

    @staticmethod
    def _tau(part, tau):
        if tau is not None:
            return float(tau)
        return {"Z": 1.0, "X": 0.0}[part]

    def sai_build(self, eps1=0.01, eps2=0.014, eps3=0.18, k_index=0, part="Z", tau=None):
        """SAI of the near field of tau R + i X at the wavenumber
        ks[k_index]: tau=1 (part="Z") Z_near, tau=0 (part="X") the real
        X_near, other tau the shifted operator of eigs(tau=...)."""
        check(lib().cm_sai_build(self._h, eps1, eps2, eps3, int(k_index), self._tau(part, tau)))

    def sai_nnz(self, part="Z", tau=None):
        """Stored entries of an SAI matrix (after sai_build; at k[0])."""
        nnz = C.c_int64()
        which = 2 if self._tau(part, tau) == 1.0 else 3
        check(lib().cm_export_near(self._h, which, C.byref(nnz), None, None, None))
        return int(nnz.value)

    def sai_apply(self, x, out=None, stream=None, k_index=None, part="Z", tau=None):
        X, Y, dt, squeeze = self._vec_args(x, out)
        ki = self._k_index(k_index, X.shape[1])
        st = lib().cm_sai_apply(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()), X.stride(0),
                                X.shape[1], None if ki is None else C.c_void_p(ki.ctypes.data),
                                self._tau(part, tau), dt, self._stream_ptr(stream))
        check(st)
        return Y.reshape(-1) if squeeze else Y

    def vdot(self, x, y, stream=None):
        """sum conj(x) * y over all entries of two (N,) or (N, ncols) CUDA
        tensors of one dtype, as a complex128 scalar tensor on the device
        (formed in the library in a fixed order; asynchronous)."""
        import torch
        X, _, dt, _ = self._vec_args(x, None)
        Y, _, dt2, _ = self._vec_args(y, None)
        if dt != dt2 or tuple(X.shape) != tuple(Y.shape):
            raise ValueError("x and y need the same dtype and shape")
        if Y.stride(0) != X.stride(0):
            X, Y = X.contiguous(), Y.contiguous()
        out = torch.empty((), dtype=torch.complex128, device=X.device)
        check(lib().cm_vdot(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()), X.stride(0), X.shape[1],
                            dt, C.c_void_p(out.data_ptr()), self._stream_ptr(stream)))
        return out

    def _modes_arg(self, J):
        import torch
        if not isinstance(J, torch.Tensor) or not J.is_cuda or J.dtype != torch.complex128:
            raise TypeError("J must be a complex128 CUDA tensor")
        J = J.reshape(-1, 1) if J.dim() == 1 else J
        if J.dim() != 2 or J.shape[0] != self.N:
            raise ValueError(f"J must have shape (N,) or (N, m) with N={self.N}")
        if J.stride(1) != 1 or J.stride(0) < J.shape[1]:
            J = J.contiguous()
        return J

    def real_currents(self, J, stream=None):
        """(Jr, R Jr): the real, R-normalised currents (Jr^T R Jr = 1) of the
        columns of J (complex128, (N, m)), as complex128 CUDA tensors with
        zero imaginary parts."""
        import torch
        J = self._modes_arg(J)
        m = J.shape[1]
        Jr = torch.empty((self.N, m), dtype=torch.complex128, device=J.device)
        RJ = torch.empty_like(Jr)
        check(lib().cm_real_currents(self._h, C.c_void_p(J.data_ptr()), J.stride(0), m, C.c_void_p(Jr.data_ptr()),
                                     C.c_void_p(RJ.data_ptr()), m, self._stream_ptr(stream)))
        return Jr, RJ

    def modal_correlation(self, Ja, Jb, stream=None):
        """|Ja^T R Jb| normalised by the R-norms of both (numpy, ma x mb), R at
        this operator's wavenumber."""
        Ja = self._modes_arg(Ja)
        Jb = self._modes_arg(Jb)
        Cm = np.zeros((Ja.shape[1], Jb.shape[1]))
        check(lib().cm_modal_correlation(self._h, C.c_void_p(Ja.data_ptr()), Ja.stride(0), Ja.shape[1],
                                         C.c_void_p(Jb.data_ptr()), Jb.stride(0), Jb.shape[1], Cm.ctypes.data,
                                         self._stream_ptr(stream)))
        return Cm

    def dlambda_dk(self, lam, J, stream=None):
        """d lambda/dk of a characteristic value (or of a degenerate cluster
        around it) from its vectors J ((N,) or (N, m) complex128); returns m
        values, ascending (cm_dlambda_dk)."""
        J = self._modes_arg(J)
        m = J.shape[1]
        d = np.zeros(m)
        check(lib().cm_dlambda_dk(self._h, float(lam), C.c_void_p(J.data_ptr()), J.stride(0), m, d.ctypes.data,
                                  self._stream_ptr(stream)))
        return d

    # ------------------------------------------------------------ Calderon preconditioner
    def cmp_build(self, nlv=0, interp_p=0, d0=0.0, stream=None):
        """Build the Calderon preconditioner of eqs. (25)-(27) (closed
        surfaces): the barycentric refinement, its MLFMA handle (nlv levels,
        0: one more than this handle's; interp_p and d0, 0: this handle's),
        the Buffa-Christiansen functions and the mixed Gram matrix
        (cm_cmp_build).  Returns dict(N_refined, B_nnz, G_nnz,
        near_nnz_refined, nlv_refined)."""
        info = np.zeros(5, dtype=np.int64)
        s = None if self.host_only else self._stream_ptr(stream)
        check(lib().cm_cmp_build(self._h, int(nlv), int(interp_p), float(d0), info.ctypes.data, s))
        return dict(N_refined=int(info[0]), B_nnz=int(info[1]), G_nnz=int(info[2]), near_nnz_refined=int(info[3]),
                    nlv_refined=int(info[4]))

    def cmp_export(self, which="G"):
        """Host copy of a Calderon table as (ptr, col, val) CSR arrays:
        which="B" (N x N_refined BC coefficients) or "G" (cm_cmp_export)."""
        if which not in ("B", "G"):
            raise ValueError("which must be 'B' or 'G'")
        w = 0 if which == "B" else 1
        rows, nnz = C.c_int64(), C.c_int64()
        check(lib().cm_cmp_export(self._h, w, C.byref(rows), C.byref(nnz), None, None, None))
        ptr = np.zeros(rows.value + 1, dtype=np.int64)
        col = np.zeros(max(1, nnz.value), dtype=np.int32)
        val = np.zeros(max(1, nnz.value))
        check(lib().cm_cmp_export(self._h, w, C.byref(rows), C.byref(nnz), ptr.ctypes.data, col.ctypes.data,
                                  val.ctypes.data))
        return ptr, col[:nnz.value], val[:nnz.value]

    def cmp_apply(self, x, which="M", far="fp64", stream=None):
        """One column through the Calderon preconditioner's matrices:
        which="Zt" Z~ x, "G" G x, "M" Z~ G^-1 Z x (cm_cmp_apply).  x: CUDA
        complex128 tensor of N."""
        import torch
        codes = {"Zt": 0, "G": 1, "M": 2}
        if which not in codes:
            raise ValueError("which must be 'Zt', 'G' or 'M'")
        if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.complex128 or x.numel() != self.N:
            raise TypeError("x must be a complex128 CUDA tensor of N entries")
        x = x.reshape(-1).contiguous()
        y = torch.empty_like(x)
        check(lib().cm_cmp_apply(self._h, codes[which], C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                 _lib.CM_C128 if far == "fp64" else _lib.CM_C64, self._stream_ptr(stream)))
        return y

    # ------------------------------------------------------------ Krylov drivers
    def gmres(self, b, restart=50, maxit=500, tol=1e-6, precond=True, far="fp64", stream=None,
              raise_on_fail=False):
        """Solve Z x = b (b: CUDA complex128 tensor of N).  precond: False,
        True (the SAI, sai_build first) or "cmp" (the Calderon preconditioner
        of eq. (25), cmp_build first; the residual is then that of
        Z~ G^-1 Z x = Z~ G^-1 b).  Returns (x, iterations, final relative
        residual, converged)."""
        import torch
        if not isinstance(b, torch.Tensor) or not b.is_cuda or b.dtype != torch.complex128 or b.numel() != self.N:
            raise TypeError("b must be a complex128 CUDA tensor of N entries")
        b = b.reshape(-1).contiguous()
        x = torch.empty_like(b)
        it = C.c_int32()
        rr = C.c_double()
        st = lib().cm_gmres(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), restart, maxit, tol,
                            _precond_code(precond), _lib.CM_C128 if far == "fp64" else _lib.CM_C64, C.byref(it),
                            C.byref(rr), self._stream_ptr(stream))
        if st not in (_lib.CM_OK, _lib.CM_E_NOT_CONVERGED) or (raise_on_fail and st != _lib.CM_OK):
            check(st)
        return x, int(it.value), float(rr.value), st == _lib.CM_OK

    def jd(self, nev, v0, target=0.0, mmin=6, mmax=20, maxit=500, tol=1e-8, inner_steps=10, precond=False,
           far="fp64", vectors=True, stream=None, harmonic=False):
        """Characteristic values closest to target by Jacobi-Davidson on the
        pencil (X, R) (no inner solve with Z).  v0: CUDA complex128 start
        vector; precond=True (or "Z") solves the corrections right-
        preconditioned by i P with the SAI P of Z (sai_build first), "X" by
        the SAI of X_near (sai_build(part="X") first); harmonic=True selects
        harmonic Ritz pairs for the target.  Returns dict(lam, resid,
        J (N x nconv, R-normalised), nconv, outer, inner_steps, n_matvec,
        precond_dropped, converged); the preconditioner is dropped after
        max(50, maxit / 8) outer iterations without a new converged pair."""
        import torch
        v0 = self._start_vector(v0)
        lam = np.zeros(nev)
        res = np.zeros(nev)
        cnt = np.zeros(4, dtype=np.int64)
        J = torch.empty((nev, self.N), dtype=torch.complex128, device=v0.device) if vectors else None
        nconv = C.c_int32()
        pc = {False: 0, None: 0, True: 1, "Z": 1, "X": 2}[precond]
        st = lib().cm_jd(self._h, nev, float(target), mmin, mmax, maxit, tol, inner_steps, pc, 1 if harmonic else 0,
                         C.c_void_p(v0.data_ptr()),
                         _lib.CM_C128 if far == "fp64" else _lib.CM_C64, lam.ctypes.data, res.ctypes.data,
                         C.c_void_p(J.data_ptr()) if vectors else None, C.byref(nconv), cnt.ctypes.data,
                         self._stream_ptr(stream))
        if st not in (_lib.CM_OK, _lib.CM_E_NOT_CONVERGED):
            check(st)
        n = int(nconv.value)
        return dict(lam=lam[:n], resid=res[:n], J=(J[:n].T if vectors else None), nconv=n, outer=int(cnt[0]),
                    inner_steps=int(cnt[1]), n_matvec=int(cnt[2]), precond_dropped=bool(cnt[3]),
                    converged=(st == _lib.CM_OK))

    def eigs(self, nev, ncv, v0, tol=1e-8, maxrestart=50, gmres_restart=50, gmres_maxit=1000, gmres_tol=1e-8,
             precond=None, far="fp64", vectors=True, stream=None, route="Z", tau=1.0):
        """Characteristic values by implicitly restarted Arnoldi on Z^-1 R.
        v0: CUDA complex128 start vector.  Returns dict(lam, resid, J, nconv,
        n_op, gmres_iters, n_matvec, restarts, inner_retries, inner_failures,
        converged); converged is False when fewer than nev Ritz values
        converged or when an inner GMRES solve missed gmres_tol.  route="X":
        IRA on X^-1 R (eq. (14)) instead of Z^-1 R, its inner solves with X
        preconditioned by the SAI of X_near when precond (sai_build(part="X")
        first).  precond=None: True for route "Z", False for route "X".
        tau (route "Z"): OP = (tau R + i X)^-1 R, tau = 1 being Z^-1 R; a
        smaller tau separates modes with |lambda| up to about tau (its SAI:
        sai_build(tau=tau)).  precond="cmp" (route "Z", tau 1): the inner
        solves take the Calderon preconditioner (cmp_build first)."""
        import torch
        v0 = self._start_vector(v0)
        lam = np.zeros(2 * nev)
        res = np.zeros(nev)
        cnt = np.zeros(6, dtype=np.int64)
        J = torch.empty((nev, self.N), dtype=torch.complex128, device=v0.device) if vectors else None
        nconv = C.c_int32()
        fd = _lib.CM_C128 if far == "fp64" else _lib.CM_C64
        Jp = C.c_void_p(J.data_ptr()) if vectors else None
        if precond is None:
            precond = route == "Z"
        if route == "X":
            st = lib().cm_eigs_xinv(self._h, nev, ncv, maxrestart, tol, C.c_void_p(v0.data_ptr()), gmres_restart,
                                    gmres_maxit, gmres_tol, 1 if precond else 0, fd, lam.ctypes.data,
                                    res.ctypes.data, Jp, C.byref(nconv), cnt.ctypes.data, self._stream_ptr(stream))
        elif route == "Z":
            st = lib().cm_eigs(self._h, nev, ncv, maxrestart, tol, C.c_void_p(v0.data_ptr()), gmres_restart,
                               gmres_maxit, gmres_tol, _precond_code(precond), float(tau), fd, lam.ctypes.data,
                               res.ctypes.data,
                               Jp, C.byref(nconv), cnt.ctypes.data, self._stream_ptr(stream))
        else:
            raise ValueError("route must be 'Z' or 'X'")
        if st not in (_lib.CM_OK, _lib.CM_E_NOT_CONVERGED):
            check(st)
        return dict(lam=lam[0::2] + 1j * lam[1::2], resid=res, J=(J.T if vectors else None), nconv=int(nconv.value),
                    n_op=int(cnt[0]), gmres_iters=int(cnt[1]), n_matvec=int(cnt[2]), restarts=int(cnt[3]),
                    inner_retries=int(cnt[4]), inner_failures=int(cnt[5]), converged=(st == _lib.CM_OK))
