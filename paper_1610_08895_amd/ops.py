"""Python handles over the C ABI: measurement operator, SARA dictionary, PD solver state.

Argument marshalling only.  Every tensor argument is checked on the host (device, dtype,
contiguity, exact shape) before anything is enqueued; all arithmetic runs in libri.so on
the current torch stream.
"""
import ctypes

import numpy as np
import torch

from . import _lib as L


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, shape, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _mask(mask, d):
    if mask is None:
        return None
    return _dev(mask, torch.uint8, (d,), "mask")


class Plan:
    """Phi = G M F Z for an n x n image, M visibilities in d blocks (Eq. 3, Eq. 8)."""

    def __init__(self, n, uv, block_off, J=8, beta=0.0, tile=0, bin=0, fft_panel=0, persistent_wgs=0,
                 slice_vis=0):
        lib = L.load()
        uv = np.ascontiguousarray(uv, dtype=np.float32)
        off = np.ascontiguousarray(block_off, dtype=np.int64)
        if uv.ndim != 2 or uv.shape[1] != 2:
            raise ValueError("uv must be (M, 2)")
        self.n, self.M, self.d = int(n), int(uv.shape[0]), int(off.size - 1)
        tune = L.Tuning(tile, bin, fft_panel, persistent_wgs, slice_vis)
        h = ctypes.c_void_p()
        L.check(lib.ri_plan_create(ctypes.byref(h), self.n, self.M, uv.ctypes.data, self.d, off.ctypes.data,
                                   J, float(beta), ctypes.byref(tune), _stream()))
        self._h = h
        K, tl, ni = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        L.check(lib.ri_plan_info(h, None, None, None, ctypes.byref(K), ctypes.byref(tl), ctypes.byref(ni)))
        self.K, self.tile, self.n_items = K.value, tl.value, ni.value
        self.block_off = off.copy()
        self.jd = 0  # DDE kernel side (set_dde); 0: plain G

    @property
    def handle(self):
        return self._h

    def set_dde(self, d):
        """Direction-dependent effects in G (ri_plan_dde): d (M, jd, jd) complex DDE kernels in
        user order, or None to remove them."""
        if d is None:
            L.check(L.load().ri_plan_dde(self._h, 0, None, _stream()))
            self.jd = 0
            return
        d = np.ascontiguousarray(d, dtype=np.complex64)
        if d.ndim != 3 or d.shape[0] != self.M or d.shape[1] != d.shape[2]:
            raise ValueError("d must be (M, jd, jd)")
        L.check(L.load().ri_plan_dde(self._h, int(d.shape[1]), d.ctypes.data, _stream()))
        self.jd = int(d.shape[1])

    def order(self):
        out = np.empty(self.M, dtype=np.int64)
        L.check(L.load().ri_plan_order(self._h, out.ctypes.data))
        return out

    def permute(self, src, to_plan=True, out=None):
        s = _dev(src, torch.complex64, (self.M,), "src")
        if out is None:
            out = torch.empty_like(src)
        L.check(L.load().ri_plan_permute(self._h, s, _dev(out, torch.complex64, (self.M,), "out"),
                                         1 if to_plan else 0, _stream()))
        return out

    def phi(self, x, y=None, mask=None):
        xp = _dev(x, torch.float32, (self.n, self.n), "x")
        if y is None:
            y = torch.zeros(self.M, dtype=torch.complex64, device=x.device)
        L.check(L.load().ri_phi(self._h, xp, _dev(y, torch.complex64, (self.M,), "y"), _mask(mask, self.d),
                                _stream()))
        return y

    def phi_adj(self, y, x=None, mask=None):
        yp = _dev(y, torch.complex64, (self.M,), "y")
        if x is None:
            x = torch.empty(self.n, self.n, dtype=torch.float32, device=y.device)
        L.check(L.load().ri_phi_adj(self._h, yp, _dev(x, torch.float32, (self.n, self.n), "x"),
                                    _mask(mask, self.d), _stream()))
        return x

    def block_sumsq(self, y, out=None):
        """||y_i||^2 per block in FP64 (device)."""
        yp = _dev(y, torch.complex64, (self.M,), "y")
        if out is None:
            out = torch.empty(self.d, dtype=torch.float64, device=y.device)
        L.check(L.load().ri_block_sumsq(self._h, yp, _dev(out, torch.float64, (self.d,), "out"), _stream()))
        return out

    def norm(self, x0, max_it=1000, rtol=1e-7):
        """||Phi||_S by power iteration from x0 (overwritten)."""
        v, it = ctypes.c_double(), ctypes.c_int()
        L.check(L.load().ri_phi_norm(self._h, _dev(x0, torch.float32, (self.n, self.n), "x0"), int(max_it),
                                     float(rtol), ctypes.byref(v), ctypes.byref(it), _stream()))
        return v.value, it.value

    def close(self):
        if getattr(self, "_h", None):
            L.load().ri_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Sara:
    """Psi: Dirac + db1..db8, `levels`-level periodic 2D DWTs (Sec. III)."""

    def __init__(self, n, levels=4, bases=0):
        lib = L.load()
        h = ctypes.c_void_p()
        L.check(lib.ri_sara_create(ctypes.byref(h), int(n), int(levels), int(bases), _stream()))
        self._h = h
        b = ctypes.c_int()
        L.check(lib.ri_sara_bases(h, ctypes.byref(b)))
        self.n, self.levels, self.b = int(n), int(levels), b.value

    @property
    def handle(self):
        return self._h

    def psi(self, s, x=None):
        sp = _dev(s, torch.float32, (self.b, self.n, self.n), "s")
        if x is None:
            x = torch.empty(self.n, self.n, dtype=torch.float32, device=s.device)
        L.check(L.load().ri_psi(self._h, sp, _dev(x, torch.float32, (self.n, self.n), "x"), _stream()))
        return x

    def psi_adj(self, x, s=None):
        xp = _dev(x, torch.float32, (self.n, self.n), "x")
        if s is None:
            s = torch.empty(self.b, self.n, self.n, dtype=torch.float32, device=x.device)
        L.check(L.load().ri_psi_adj(self._h, xp, _dev(s, torch.float32, (self.b, self.n, self.n), "s"),
                                    _stream()))
        return s

    def norm(self, x0, max_it=1000, rtol=1e-7):
        v, it = ctypes.c_double(), ctypes.c_int()
        L.check(L.load().ri_psi_norm(self._h, _dev(x0, torch.float32, (self.n, self.n), "x0"), int(max_it),
                                     float(rtol), ctypes.byref(v), ctypes.byref(it), _stream()))
        return v.value, it.value

    def close(self):
        if getattr(self, "_h", None):
            L.load().ri_sara_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PD:
    """State of Algorithm 1 on the GPU (x, x~, s, v and the running sum of v~)."""

    def __init__(self, plan: Plan, sara: Sara, y, eps, tau, sigma, varsigma, kappa, psi_norm, phi_norm):
        lib = L.load()
        self.plan, self.sara = plan, sara
        yp = _dev(y, torch.complex64, (plan.M,), "y")
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        if eps.shape != (plan.d,):
            raise ValueError("eps must have one radius per block")
        prm = L.PDParams(tau, sigma, varsigma, kappa, psi_norm, phi_norm)
        h = ctypes.c_void_p()
        L.check(lib.ri_pd_create(ctypes.byref(h), plan.handle, sara.handle, yp, eps.ctypes.data,
                                 ctypes.byref(prm), _stream()))
        self._h = h
        self.eps = eps
        self.params = dict(tau=tau, sigma=sigma, varsigma=varsigma, kappa=kappa, psi_norm=psi_norm,
                           phi_norm=phi_norm)

    def step(self, mask=None, stats=None):
        st = None if stats is None else _dev(stats, torch.float64, (self.plan.d, 2), "stats")
        L.check(L.load().ri_pd_step(self._h, _mask(mask, self.plan.d), st, _stream()))

    def step_plain(self, mask_host=None, stats=None):
        mh = None
        if mask_host is not None:
            mh = np.ascontiguousarray(mask_host, dtype=np.uint8)
            if mh.shape != (self.plan.d,):
                raise ValueError("mask_host must have d entries")
        st = None if stats is None else _dev(stats, torch.float64, (self.plan.d, 2), "stats")
        L.check(L.load().ri_pd_step_plain(self._h, None if mh is None else mh.ctypes.data, st, _stream()))

    def refresh(self):
        L.check(L.load().ri_pd_refresh(self._h, _stream()))

    def residual(self, out=None):
        """(d, 2) FP64 device tensor; column 1 holds ||Phi_i x - y_i||^2 at the current x for
        every block (ri_pd_residual), column 0 ||v_i + Phi_i x - y_i||^2."""
        if out is None:
            out = torch.empty(self.plan.d, 2, dtype=torch.float64, device="cuda")
        L.check(L.load().ri_pd_residual(self._h, _dev(out, torch.float64, (self.plan.d, 2), "out"), _stream()))
        return out

    def step_vjp(self, mask, x_new, s_new, v_new, r, stats, xbar, xtbar, sbar, vbar, pgrad):
        """Reverse sweep of one step (ri_pd_step_vjp): the adjoints xbar, xtbar, sbar, vbar
        are updated in place from after the step to before it; pgrad (2 FP64) accumulates
        the step's dL/dtau and dL/dsigma."""
        n, b, M, d = self.plan.n, self.sara.b, self.plan.M, self.plan.d
        L.check(L.load().ri_pd_step_vjp(
            self._h, _mask(mask, d), _dev(x_new, torch.float32, (n, n), "x_new"),
            _dev(s_new, torch.float32, (b, n, n), "s_new"), _dev(v_new, torch.complex64, (M,), "v_new"),
            _dev(r, torch.complex64, (M,), "r"),
            _dev(stats, torch.float64, (d, 2), "stats"), _dev(xbar, torch.float32, (n, n), "xbar"),
            _dev(xtbar, torch.float32, (n, n), "xtbar"), _dev(sbar, torch.float32, (b, n, n), "sbar"),
            _dev(vbar, torch.complex64, (M,), "vbar"), _dev(pgrad, torch.float64, (2,), "pgrad"), _stream()))

    def timing(self, enable=True):
        """Record a HIP event pair around every stage of the following steps."""
        L.check(L.load().ri_pd_timing(self._h, 1 if enable else 0))

    def stage_times(self):
        """{stage: (total ms, launches)} since timing was enabled; clears the records."""
        n = len(L.STAGES)
        tot = np.zeros(n)
        cnt = np.zeros(n, dtype=np.int32)
        L.check(L.load().ri_pd_stage_times(self._h, tot.ctypes.data, cnt.ctypes.data, n))
        return {name: (float(tot[i]), int(cnt[i])) for i, name in enumerate(L.STAGES)}

    def reweight(self, delta):
        """Weights w = delta / (delta + |Psi^dagger x|) of the weighted l1 prior, from the
        current x (ri_pd_reweight); later steps clip at alpha w."""
        L.check(L.load().ri_pd_reweight(self._h, float(delta), _stream()))

    @property
    def weighted(self):
        v = ctypes.c_int()
        L.check(L.load().ri_pd_weighted(self._h, ctypes.byref(v)))
        return bool(v.value)

    def unweight(self):
        """Back to the plain l1 prior."""
        L.check(L.load().ri_pd_set(self._h, L.RI_PD_W, None, 0, _stream()))

    def _shape(self, which):
        n = self.plan.n
        return {L.RI_PD_X: ((n, n), torch.float32), L.RI_PD_XTILDE: ((n, n), torch.float32),
                L.RI_PD_S: ((self.sara.b, n, n), torch.float32), L.RI_PD_W: ((self.sara.b, n, n), torch.float32),
                L.RI_PD_V: ((self.plan.M,), torch.complex64), L.RI_PD_E: ((self.plan.M,), torch.complex64)}[which]

    def get(self, which, out=None):
        shape, dt = self._shape(which)
        if out is None:
            out = torch.empty(shape, dtype=dt, device="cuda")
        p = _dev(out, dt, shape, "out")
        L.check(L.load().ri_pd_get(self._h, which, p, out.numel() * out.element_size(), _stream()))
        return out

    def set(self, which, value):
        shape, dt = self._shape(which)
        p = _dev(value, dt, shape, "value")
        L.check(L.load().ri_pd_set(self._h, which, p, value.numel() * value.element_size(), _stream()))

    @property
    def iteration(self):
        v = ctypes.c_int64()
        L.check(L.load().ri_pd_get(self._h, L.RI_PD_ITER, ctypes.byref(v), 8, None))
        return v.value

    @iteration.setter
    def iteration(self, t):
        v = ctypes.c_int64(int(t))
        L.check(L.load().ri_pd_set(self._h, L.RI_PD_ITER, ctypes.byref(v), 8, None))

    def close(self):
        if getattr(self, "_h", None):
            L.load().ri_pd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceSchedule:
    """Buffers of the device-side block selection (ri_sched_step) for T iterations.

    Exactly one of u (T x d uniforms, drawn against the probabilities) or masks (T x d,
    replayed) is given.  p_fixed: d probabilities of a non-adaptive schedule (None: 1).
    c0: the Eq. 13 energies at the start of an adaptive run.  stats_step, stats_x: the
    (d, 2) FP64 device tensors that ri_pd_step and ri_pd_residual write.  The mask tensor
    is what the step reads; p_log and mask_log keep every iteration's probabilities and
    mask on the device until read back.
    """

    def __init__(self, d, T, eps, stats_step, stats_x=None, u=None, masks=None, p_fixed=None, c0=None,
                 n_nodes=0.0, p_min=0.05, p_max=0.5):
        if (u is None) == (masks is None):
            raise ValueError("give exactly one of u and masks")
        dev = "cuda"
        self.d, self.T = int(d), int(T)
        f64 = dict(dtype=torch.float64, device=dev)
        self.u = None if u is None else torch.tensor(np.asarray(u, np.float64).reshape(T, d), **f64)
        self.masks = None if masks is None else torch.tensor(np.asarray(masks, np.uint8).reshape(T, d),
                                                              dtype=torch.uint8, device=dev)
        self.p_fixed = None if p_fixed is None else torch.tensor(np.asarray(p_fixed, np.float64).reshape(d), **f64)
        self.c = torch.tensor(np.zeros(d) if c0 is None else np.asarray(c0, np.float64).reshape(d), **f64)
        self.eps = torch.tensor(np.asarray(eps, np.float64).reshape(d), **f64)
        self.counter = torch.zeros(1, dtype=torch.int64, device=dev)
        self.mask = torch.ones(d, dtype=torch.uint8, device=dev)
        self.p_log = torch.zeros(T, d, **f64)
        self.mask_log = torch.zeros(T, d, dtype=torch.uint8, device=dev)
        _dev(stats_step, torch.float64, (d, 2), "stats_step")
        if stats_x is not None:
            _dev(stats_x, torch.float64, (d, 2), "stats_x")
        self.stats_step, self.stats_x = stats_step, stats_x

        def ptr(t):
            return None if t is None else t.data_ptr()

        self._a = L.Sched(self.d, self.T, ptr(self.u), ptr(self.masks), ptr(self.p_fixed), ptr(self.c),
                          ptr(stats_step), ptr(stats_x), ptr(self.eps), float(n_nodes), float(p_min),
                          float(p_max), ptr(self.counter), ptr(self.mask), ptr(self.p_log), ptr(self.mask_log))

    def step(self, flags):
        L.check(L.load().ri_sched_step(ctypes.byref(self._a), int(flags), _stream()))


def residual_energy(resid_norm, eps):
    """Eq. 13 (host, in the library)."""
    r = np.ascontiguousarray(resid_norm, dtype=np.float64)
    e = np.ascontiguousarray(eps, dtype=np.float64)
    out = np.empty_like(r)
    L.check(L.load().ri_residual_energy(r.ctypes.data, e.ctypes.data, r.size, out.ctypes.data))
    return out


def probabilities(c, n_nodes, p_min, p_max):
    """Eq. 14 (host, in the library).  Returns (p, a)."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    p = np.empty_like(c)
    a = ctypes.c_double()
    L.check(L.load().ri_probs(c.ctypes.data, c.size, float(n_nodes), float(p_min), float(p_max), p.ctypes.data,
                              ctypes.byref(a)))
    return p, a.value
