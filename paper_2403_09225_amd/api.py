"""Python binding of the PWA likelihood library: argument marshalling only.

torch provides device memory and the stream; every step of the evaluation
runs in the library's HIP kernels.

    lik = Likelihood(channel=[0, 0], spin=[0, 1])
    lik.bind(data_s12, data_s13, mc_s12, mc_s13)      # tensors or arrays
    nll = lik.nll(theta)                              # theta: float64 (4K,)
    nll, g = lik.grad(theta)
    hv, nll, g = lik.hvp(theta, v)
    theta_fit, report = lik.fit(theta0, xtol=1e-8)
"""

import ctypes

import numpy as np
import torch

from . import _lib as L

PARENT_MASS = 1.865
DAUGHTER_MASSES = (0.494, 0.140, 0.140)
R_BARRIER = 3.0


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev_f64(x, device):
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=torch.float64).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device=device)


class Likelihood:
    """Unbinned PWA NLL, gradient and Hessian-vector product on one GPU."""

    def __init__(self, channel, spin, parent_mass=PARENT_MASS, masses=DAUGHTER_MASSES,
                 r=R_BARRIER, width_mode=0, streams=("f64",), device="cuda", lineshape=None,
                 flatte_masses=(0.0, 0.0), flatte_ratio=0.0, parent_spin=0):
        """lineshape: per resonance 0 (Breit-Wigner) or 1 (Flatte, J = 0;
        theta[4k+3] is then g_1), with the second channel's masses and the
        coupling ratio g_2 / g_1; parent_spin 1: a vector parent (events carry
        their orientation, see bind_oriented)."""
        self.lib = L.load()
        m = L.PwaModel()
        m.parent_mass = parent_mass
        for i in range(3):
            m.masses[i] = masses[i]
        m.r = r
        m.n_res = len(channel)
        m.width_mode = width_mode
        if len(channel) > L.PWA_MAX_RES or len(spin) != len(channel):
            raise ValueError("channel/spin lists must have equal length <= 64")
        for k, (c, j) in enumerate(zip(channel, spin)):
            m.channel[k] = int(c)
            m.spin[k] = int(j)
            m.lineshape[k] = int(lineshape[k]) if lineshape is not None else 0
        m.flatte_masses[0], m.flatte_masses[1] = flatte_masses
        m.flatte_ratio = flatte_ratio
        m.parent_spin = parent_spin
        self.parent_spin = parent_spin
        mask = (L.PWA_STREAM_F64 if "f64" in streams else 0) | (L.PWA_STREAM_F32 if "f32" in streams else 0)
        h = ctypes.c_void_p()
        L.check("pwa_create", self.lib.pwa_create(ctypes.byref(m), mask, ctypes.byref(h)))
        self._h = h
        self.n_res = len(channel)
        self.n_par = 4 * self.n_res
        self.device = torch.device(device)
        self.streams = tuple(streams)
        self._ws = None
        self.n_data = self.n_mc = 0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.lib.pwa_destroy(h)
            self._h = None

    # ---------------------------------------------------------------- binding
    def workspace_bytes(self, n_data, n_mc):
        return int(self.lib.pwa_workspace_bytes(self._h, int(n_data), int(n_mc)))

    def _workspace(self, nd, nm):
        nbytes = self.workspace_bytes(nd, nm)
        if nbytes == 0:
            raise ValueError("invalid event counts")
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-ws.data_ptr()) % 256
        self._ws = ws
        return ctypes.c_void_p(ws.data_ptr() + off), nbytes

    def bind(self, data_s12, data_s13, mc_s12, mc_s13):
        """Copy events to the device (if needed) and build the event stream."""
        d12, d13 = _dev_f64(data_s12, self.device), _dev_f64(data_s13, self.device)
        m12, m13 = _dev_f64(mc_s12, self.device), _dev_f64(mc_s13, self.device)
        nd, nm = int(d12.numel()), int(m12.numel())
        wptr, nbytes = self._workspace(nd, nm)
        L.check("pwa_bind", self.lib.pwa_bind(
            self._h, _ptr(d12) if nd else None, _ptr(d13) if nd else None, nd,
            _ptr(m12), _ptr(m13), nm, wptr, nbytes, _stream()))
        torch.cuda.current_stream().synchronize()  # event arrays may be freed now
        self.n_data, self.n_mc = nd, nm
        return self

    def bind_oriented(self, data, mc):
        """bind for a spin-1 parent: data and mc are (s12, s13, cos_beta,
        gamma) tuples of arrays or tensors."""
        d = [_dev_f64(x, self.device) for x in data]
        m = [_dev_f64(x, self.device) for x in mc]
        nd, nm = int(d[0].numel()), int(m[0].numel())
        wptr, nbytes = self._workspace(nd, nm)
        dp = [_ptr(x) if nd else None for x in d]
        L.check("pwa_bind_oriented", self.lib.pwa_bind_oriented(
            self._h, dp[0], dp[1], dp[2], dp[3], nd, _ptr(m[0]), _ptr(m[1]), _ptr(m[2]), _ptr(m[3]),
            nm, wptr, nbytes, _stream()))
        torch.cuda.current_stream().synchronize()
        self.n_data, self.n_mc = nd, nm
        return self

    def set_precision(self, prec):
        L.check("pwa_set_precision", self.lib.pwa_set_precision(
            self._h, L.PWA_PREC_F32 if prec == "f32" else L.PWA_PREC_F64))

    def set_launch_shape(self, layout=0, groups=0, res_per_group=0):
        """layout 1: `groups` lanes per event; layout 2: `groups` waves per 64
        events; layout 3: the same for the general physics path; 0:
        automatic."""
        L.check("pwa_set_launch_shape",
                self.lib.pwa_set_launch_shape(self._h, layout, groups, res_per_group))

    def grid_blocks(self):
        return int(self.lib.pwa_grid_blocks(self._h))

    def stream_fields(self):
        """Per-event planes of the event stream (8 bytes each per event on the
        FP64 stream, 4 on the FP32 one)."""
        return int(self.lib.pwa_stream_fields(self._h))

    def set_kernel_timing(self, enable=True):
        L.check("pwa_set_kernel_timing", self.lib.pwa_set_kernel_timing(self._h, 1 if enable else 0))

    def kernel_time(self):
        """(summed ms, launches) of the per-event pass kernel since the last call."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        L.check("pwa_kernel_time", self.lib.pwa_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    # ------------------------------------------------------------ evaluation
    def _theta(self, theta):
        t = _dev_f64(theta, self.device)
        if t.numel() != self.n_par:
            raise ValueError(f"theta must have {self.n_par} entries")
        return t

    def nll(self, theta):
        t = self._theta(theta)
        out = torch.empty((), dtype=torch.float64, device=self.device)
        L.check("pwa_nll", self.lib.pwa_nll(self._h, _ptr(t), _ptr(out), _stream()))
        return out

    def grad(self, theta):
        t = self._theta(theta)
        out = torch.empty(1 + self.n_par, dtype=torch.float64, device=self.device)
        L.check("pwa_grad", self.lib.pwa_grad(
            self._h, _ptr(t), _ptr(out), ctypes.c_void_p(out.data_ptr() + 8), _stream()))
        return out[0], out[1:]

    def hvp(self, theta, v):
        t = self._theta(theta)
        vv = self._theta(v)
        out = torch.empty(1 + 2 * self.n_par, dtype=torch.float64, device=self.device)
        base = out.data_ptr()
        L.check("pwa_hvp", self.lib.pwa_hvp(
            self._h, _ptr(t), _ptr(vv), ctypes.c_void_p(base + 8 * (1 + self.n_par)),
            ctypes.c_void_p(base), ctypes.c_void_p(base + 8), _stream()))
        return out[1 + self.n_par:], out[0], out[1:1 + self.n_par]

    def hvp_reuse(self, v):
        """H v at the theta of the last hvp() call (direction-only pass);
        returns (hv, nll, grad) like hvp()."""
        vv = self._theta(v)
        out = torch.empty(1 + 2 * self.n_par, dtype=torch.float64, device=self.device)
        base = out.data_ptr()
        L.check("pwa_hvp_reuse", self.lib.pwa_hvp_reuse(
            self._h, _ptr(vv), ctypes.c_void_p(base + 8 * (1 + self.n_par)),
            ctypes.c_void_p(base), ctypes.c_void_p(base + 8), _stream()))
        return out[1 + self.n_par:], out[0], out[1:1 + self.n_par]

    def intensity(self, theta, which="data"):
        """Per-event omega(x) at theta for the bound data or MC events (eq. (1))."""
        t = self._theta(theta)
        w = {"data": 0, "mc": 1}[which]
        n = self.n_data if w == 0 else self.n_mc
        out = torch.empty(n, dtype=torch.float64, device=self.device)
        L.check("pwa_intensity", self.lib.pwa_intensity(self._h, _ptr(t), w, _ptr(out), _stream()))
        return out

    def partials(self, theta, v=None):
        """(hi, lo) pairs of [F, G, dF, dG, H_F v, H_G v] (eq. (5) and derivatives)."""
        t = self._theta(theta)
        vv = self._theta(v) if v is not None else None
        out = torch.empty(2 * (2 + 4 * self.n_par), dtype=torch.float64, device=self.device)
        L.check("pwa_partials", self.lib.pwa_partials(self._h, _ptr(t), _ptr(vv), _ptr(out), _stream()))
        return out

    def partials_reuse(self, v):
        """partials() with a new direction at the theta of the last
        hvp()/partials(theta, v) call (direction-only pass)."""
        vv = self._theta(v)
        out = torch.empty(2 * (2 + 4 * self.n_par), dtype=torch.float64, device=self.device)
        L.check("pwa_partials_reuse", self.lib.pwa_partials_reuse(self._h, _ptr(vv), _ptr(out), _stream()))
        return out

    def combine(self, parts, n_data_total, n_mc_total, v=None):
        return combine(parts, self.n_par, n_data_total, n_mc_total, v, self.device)

    def device_status(self):
        s = self.lib.pwa_device_status(self._h, _stream())
        if s < 0:
            L.check("pwa_device_status", s)
        return s

    # ----------------------------------------------------- batched path
    def freeze(self, theta, operand="f32", max_batch=256):
        """Freeze M and Gamma at theta and build the batched-path operands."""
        t = self._theta(theta)
        fmt = L.OPERANDS[operand]
        nbytes = int(self.lib.pwa_batched_workspace_bytes(self._h, self.n_data, fmt, max_batch))
        if nbytes == 0:
            raise ValueError("batched path unavailable for these arguments (K <= 24)")
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-ws.data_ptr()) % 256
        self._bws = ws
        L.check("pwa_freeze", self.lib.pwa_freeze(
            self._h, _ptr(t), fmt, max_batch, ctypes.c_void_p(ws.data_ptr() + off), nbytes, _stream()))
        self._t_frozen = t
        return self

    def nll_batched(self, C):
        """NLL for every column of the complex K x B coupling matrix C."""
        if isinstance(C, torch.Tensor):
            Cc = C.to(self.device)
        else:
            Cc = torch.as_tensor(np.asarray(C), device=self.device)
        B = Cc.shape[1]
        ri = torch.view_as_real(Cc.to(torch.complex128).T.contiguous()).contiguous()  # (B, K, 2)
        out = torch.empty(B, dtype=torch.float64, device=self.device)
        L.check("pwa_nll_batched", self.lib.pwa_nll_batched(self._h, _ptr(ri), B, _ptr(out), _stream()))
        self._C_keep = ri
        return out

    def gram(self):
        out = torch.empty(2 * self.n_res * self.n_res, dtype=torch.float64, device=self.device)
        L.check("pwa_gram", self.lib.pwa_gram(self._h, _ptr(out), _stream()))
        return torch.view_as_complex(out.view(self.n_res, self.n_res, 2))

    # ------------------------------------------------------ at the minimum
    def hessian(self, theta):
        """Symmetrised P x P Hessian of the NLL (P Hessian-vector passes)."""
        t = self._theta(theta)
        out = torch.empty((self.n_par, self.n_par), dtype=torch.float64, device=self.device)
        L.check("pwa_hessian", self.lib.pwa_hessian(self._h, _ptr(t), _ptr(out), _stream()))
        return out

    def fit_fractions(self, theta, with_grad=True):
        """F_k = sum_MC |c_k a_k|^2 / sum_MC |z|^2 and (with_grad) dF_k/dtheta (K x P)."""
        t = self._theta(theta)
        ff = torch.empty(self.n_res, dtype=torch.float64, device=self.device)
        dff = (torch.empty((self.n_res, self.n_par), dtype=torch.float64, device=self.device)
               if with_grad else None)
        L.check("pwa_fit_fractions", self.lib.pwa_fit_fractions(
            self._h, _ptr(t), _ptr(ff), _ptr(dff), _stream()))
        return (ff, dff) if with_grad else ff

    def fraction_matrix(self, theta):
        """K x K matrix: fit fractions on the diagonal, interference terms
        I_kl above it (k < l), zero below; the entries add up to 1 (K <= 24)."""
        t = self._theta(theta)
        nbytes = int(self.lib.pwa_fraction_matrix_workspace_bytes(self._h))
        if nbytes == 0:
            raise ValueError("fraction matrix needs K <= 24 and the FP64 event stream")
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-ws.data_ptr()) % 256
        out = torch.empty((self.n_res, self.n_res), dtype=torch.float64, device=self.device)
        L.check("pwa_fraction_matrix", self.lib.pwa_fraction_matrix(
            self._h, _ptr(t), ctypes.c_void_p(ws.data_ptr() + off), nbytes, _ptr(out), _stream()))
        torch.cuda.current_stream().synchronize()   # ws is released on return
        return out

    def errors(self, theta, free_mask=None):
        """Covariance of the free parameters, parameter errors, fit fractions
        and their propagated errors at theta (normally a fitted minimum).
        Returns a dict of host arrays."""
        H = self.hessian(theta)
        ff, dff = self.fit_fractions(theta)
        return errors_from(H.cpu().numpy(), ff.cpu().numpy(), dff.cpu().numpy(), free_mask)

    # ------------------------------------------------------------------- fit
    def fit(self, theta0, xtol=1e-8, maxiter=200, cg_maxiter=0, time_cap_s=0.0,
            hvp_precision="f64", free_mask=None, forcing="scipy", precondition=False,
            method="newton-cg", reconjugate=False):
        """Newton-CG fit from theta0 (method="bfgs": the gradient-only BFGS
        comparator, pwa_fit_bfgs); returns (theta, report dict).
        forcing: "scipy" (eta = min(1/2, sqrt(sum|g|))) or "relative"
        (eta = min(1/2, sqrt(sum|g| / sum|g_0|))).  precondition: CG with
        the inverse of |H| built from HVPs; reconjugate: CG directions kept
        H-conjugate to all earlier ones of a solve (see pwa_fit_opts)."""
        entry = {"newton-cg": self.lib.pwa_fit, "bfgs": self.lib.pwa_fit_bfgs}[method]
        t = self._theta(theta0).clone()
        o = L.PwaFitOpts()
        o.xtol = xtol
        o.maxiter = maxiter
        o.cg_maxiter = cg_maxiter
        o.time_cap_s = time_cap_s
        o.hvp_precision = L.PWA_PREC_F32 if hvp_precision == "f32" else L.PWA_PREC_F64
        o.forcing = {"scipy": 0, "relative": 1}[forcing]
        o.precondition = 1 if precondition else 0
        o.reconjugate = 1 if reconjugate else 0
        o.free_mask_set = 0 if free_mask is None else 1
        if free_mask is not None:
            for i, f in enumerate(free_mask):
                o.free_mask[i] = 1 if f else 0
        rep = L.PwaFitReport()
        code = entry(self._h, _ptr(t), ctypes.byref(o), ctypes.byref(rep), _stream())
        if code not in (L.PWA_OK, L.PWA_E_NOCONV, L.PWA_E_DOMAIN):
            L.check(entry.__name__, code)
        report = {f: getattr(rep, f) for f, _ in L.PwaFitReport._fields_}
        report["code"] = int(code)
        return t, report


def combine(parts, n_par, n_data_total, n_mc_total, v=None, device="cuda"):
    """Eq. (4), (6), (7) over shard partials (list of pwa_partials outputs)."""
    lib = L.load()
    stacked = torch.cat([p.reshape(-1) for p in parts]).contiguous()
    out = torch.empty(1 + 2 * n_par, dtype=torch.float64, device=device)
    base = out.data_ptr()
    vv = _dev_f64(v, device) if v is not None else None
    L.check("pwa_combine", lib.pwa_combine(
        n_par, len(parts), _ptr(stacked), int(n_data_total), int(n_mc_total), _ptr(vv),
        ctypes.c_void_p(base), ctypes.c_void_p(base + 8),
        ctypes.c_void_p(base + 8 * (1 + n_par)) if v is not None else None, _stream()))
    return out[0], out[1:1 + n_par], (out[1 + n_par:] if v is not None else None)


def covariance(H, free_mask=None):
    """Inverse of the Hessian's free block (pwa_covariance); host arrays."""
    lib = L.load()
    H = np.ascontiguousarray(H, dtype=np.float64)
    P = H.shape[0]
    cov = np.empty((P, P))
    fm = None
    if free_mask is not None:
        fm = np.ascontiguousarray(np.asarray(free_mask, dtype=bool), dtype=np.uint8)
    L.check("pwa_covariance", lib.pwa_covariance(
        P, H.ctypes.data_as(ctypes.c_void_p),
        fm.ctypes.data_as(ctypes.c_void_p) if fm is not None else None,
        cov.ctypes.data_as(ctypes.c_void_p)))
    return cov


def propagate(J, cov):
    """sigma_r = sqrt(J_r C J_r^T) for the rows of J (pwa_propagate)."""
    lib = L.load()
    J = np.ascontiguousarray(np.atleast_2d(J), dtype=np.float64)
    cov = np.ascontiguousarray(cov, dtype=np.float64)
    sig = np.empty(J.shape[0])
    L.check("pwa_propagate", lib.pwa_propagate(
        cov.shape[0], J.shape[0], J.ctypes.data_as(ctypes.c_void_p),
        cov.ctypes.data_as(ctypes.c_void_p), sig.ctypes.data_as(ctypes.c_void_p)))
    return sig


def errors_from(H, ff, dff, free_mask=None):
    cov = covariance(H, free_mask)
    return {"hessian": H, "covariance": cov, "sigma": np.sqrt(np.clip(np.diag(cov), 0, None)),
            "fit_fractions": ff, "fit_fraction_sigma": propagate(dff, cov)}
