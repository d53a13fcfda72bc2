"""Tensor-level wrappers of the C ABI (argument marshalling only).

Every function here hands device pointers of torch tensors to libapx.so and returns
the tensors the library filled.  Parameter objects are duck-typed: any object with the
attribute names of the corresponding apx.h structure works.
"""

from __future__ import annotations

import ctypes as C
import dataclasses

import numpy as np
import torch

from . import binding as B


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """An apx_ctx bound to a device; every call enqueues on torch's current stream."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required")
        self.lib = B.load()
        self.device = device
        self.torch_device = torch.device("cuda", device)
        h = C.c_void_p()
        stream = torch.cuda.current_stream(self.torch_device).cuda_stream
        self._check(self.lib.apx_ctx_create(device, C.c_void_p(stream), C.byref(h)), h)
        self.h = h

    def _check(self, code, h=None):
        if code != B.APX_OK:
            msg = self.lib.apx_last_error(h if h is not None else self.h)
            raise B.ApxError(code, (msg or b"").decode())

    def bind_stream(self):
        s = torch.cuda.current_stream(self.torch_device).cuda_stream
        self.lib.apx_ctx_set_stream(self.h, C.c_void_p(s))

    def profile(self, on: bool = True):
        """Enables (and resets) per-kernel event timing."""
        self._check(self.lib.apx_profile_enable(self.h, 1 if on else 0))

    def profile_read(self) -> dict:
        """{kernel: (launches, total_ms)} accumulated since profile() (synchronises)."""
        k = self.lib.apx_profile_count(self.h)
        if k < 0:
            self._check(k)
        out = {}
        for e in range(k):
            name = C.c_char_p()
            launches = C.c_int64()
            ms = C.c_double()
            self._check(self.lib.apx_profile_entry(self.h, e, C.byref(name), C.byref(launches), C.byref(ms)))
            out[name.value.decode()] = (int(launches.value), float(ms.value))
        return out

    def close(self):
        if getattr(self, "h", None):
            self.lib.apx_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclasses.dataclass
class DeviceAtoms:
    pos: torch.Tensor  # [3, n] float64 cuda
    lo: tuple
    hi: tuple
    periodic: tuple
    frozen: torch.Tensor | None = None  # [n] uint8 cuda

    @property
    def n(self) -> int:
        return int(self.pos.shape[1])

    def struct(self) -> B.Atoms:
        a = B.Atoms()
        a.n = self.n
        a.pos = self.pos.data_ptr() if self.n else None
        for d in range(3):
            a.lo[d] = float(self.lo[d])
            a.hi[d] = float(self.hi[d])
            a.periodic[d] = int(bool(self.periodic[d]))
        a.frozen = None if self.frozen is None else self.frozen.data_ptr()
        return a


def device_atoms(system, device="cuda") -> DeviceAtoms:
    """Copies a host configuration (``pos`` [3, n], ``lo``, ``hi``, ``periodic``, ``frozen``)."""
    pos = torch.as_tensor(np.ascontiguousarray(system.pos), dtype=torch.float64).to(device).contiguous()
    frozen = None
    if getattr(system, "frozen", None) is not None:
        frozen = torch.as_tensor(np.ascontiguousarray(system.frozen, dtype=np.uint8)).to(device)
    return DeviceAtoms(pos, tuple(map(float, system.lo)), tuple(map(float, system.hi)),
                       tuple(int(p) for p in system.periodic), frozen)


@dataclasses.dataclass
class NeighborList:
    count: torch.Tensor  # [n] int32
    idx: torch.Tensor  # [max_nb, n] int32
    max_nb: int
    r_list: float
    needed: int = 0

    def struct(self) -> B.NList:
        s = B.NList()
        s.n = int(self.count.shape[0])
        s.max_nb = int(self.max_nb)
        s.count = self.count.data_ptr() if s.n else None
        s.idx = self.idx.data_ptr() if s.n else None
        s.r_list = float(self.r_list)
        return s


def build_neighbors(ctx: Context, atoms: DeviceAtoms, r_list: float, max_nb: int = 80,
                    grow: bool = True) -> NeighborList:
    """apx_build_neighbors; with ``grow`` a too-small capacity is enlarged once."""
    ctx.bind_stream()
    n = atoms.n
    for attempt in range(2):
        count = torch.empty(n, dtype=torch.int32, device=atoms.pos.device)
        idx = torch.empty((max_nb, n), dtype=torch.int32, device=atoms.pos.device)
        nl = NeighborList(count, idx, max_nb, r_list)
        st = nl.struct()
        a = atoms.struct()
        needed = C.c_int32(0)
        code = ctx.lib.apx_build_neighbors(ctx.h, C.byref(a), float(r_list), C.byref(st), C.byref(needed))
        nl.needed = int(needed.value)
        if code == B.APX_ECAPACITY and grow and attempt == 0 and nl.needed <= 128:
            max_nb = nl.needed
            continue
        ctx._check(code)
        return nl
    raise RuntimeError("unreachable")


def prec_struct(p, csp_given: bool = False) -> B.PrecParams:
    s = B.PrecParams()
    s.flags = (B.APX_PREC_CSP_GIVEN if csp_given else 0) | \
        (B.APX_PREC_EXTRA_LOCAL if getattr(p, "extra_local", False) else 0)
    s.n_nn = int(getattr(p, "n_nn", 12))
    s.n_buffer = int(getattr(p, "n_buffer", 0))
    s.switch_kind = int(p.switch_kind)
    s.csp_lo = float(p.csp_lo)
    s.csp_hi = float(p.csp_hi)
    s.r_cut = float(getattr(p, "r_cut", 5.0))
    s.r_lo = float(getattr(p, "r_lo", 0.0))
    s.r_hi = float(getattr(p, "r_hi", 0.0))
    return s


def eam_struct(p) -> B.EamParams:
    """apx_eam_params of a closed-form parameter object, or of an EAM2 one (field ``xi0``)."""
    s = B.EamParams()
    s.r_cut = float(getattr(p, "rc", getattr(p, "r_cut", 5.0)))
    s.h = float(p.h)
    if hasattr(p, "xi0"):
        s.kind = B.EAM2
        vals = [p.E1, p.E2, p.delta, p.alpha1, p.alpha2, p.r01, p.r02, *p.S, *p.rs, p.a, p.beta1, p.beta2, p.r03,
                p.r04, p.xi0, p.xi2, *p.q, p.Q1, p.Q2, p.f0]
        assert len(vals) == 27
        for k, v in enumerate(vals):
            s.eam2[k] = float(v)
        return s
    s.kind = B.EAM_CLOSED
    s.A, s.alpha, s.beta, s.r0 = float(p.A), float(p.alpha), float(p.beta), float(p.r0)
    return s


def compute_precision(ctx: Context, atoms: DeviceAtoms, nl: NeighborList, params, w0_extra=None,
                      csp=None) -> dict:
    """apx_compute_precision; with ``csp`` given the CSP pass is skipped and it is used."""
    ctx.bind_stream()
    n = atoms.n
    dev = atoms.pos.device
    out = dict(csp=csp if csp is not None else torch.empty(n, dtype=torch.float64, device=dev),
               w0=torch.empty(n, dtype=torch.float64, device=dev),
               w=torch.empty(n, dtype=torch.float64, device=dev),
               mask=torch.empty(n, dtype=torch.uint8, device=dev),
               active=torch.empty(max(n, 1), dtype=torch.int32, device=dev))
    na = C.c_int64(0)
    a, s, pp = atoms.struct(), nl.struct(), prec_struct(params, csp is not None)
    ctx._check(ctx.lib.apx_compute_precision(ctx.h, C.byref(a), C.byref(s), C.byref(pp), _p(w0_extra),
                                             _p(out["csp"]), _p(out["w0"]), _p(out["w"]), _p(out["mask"]),
                                             _p(out["active"]), C.byref(na)))
    out["n_active"] = int(na.value)
    out["active"] = out["active"][: out["n_active"]]
    return out


class TimeAveragedSwitch:
    """State of apx_compute_precision_avg: the CSP and spread-weight rings [n_avg][n], the
    sample counter and the filtered weight w (kept between calls)."""

    def __init__(self, n: int, n_avg: int, dw_min: float, device="cuda", window: str = "past"):
        self.n, self.n_avg, self.dw_min = int(n), int(n_avg), float(dw_min)
        self.window = {"past": B.WINDOW_PAST, "current": B.WINDOW_CURRENT}[window]
        self.csp_ring = torch.zeros((self.n_avg, self.n), dtype=torch.float64, device=device)
        self.w_ring = torch.zeros((self.n_avg, self.n), dtype=torch.float64, device=device)
        self.w = torch.zeros(self.n, dtype=torch.float64, device=device)
        self.samples = 0

    def update(self, ctx: Context, atoms: DeviceAtoms, nl: NeighborList, params, w0_extra=None,
               csp=None) -> dict:
        """One sample at the positions of ``atoms``; ``csp`` given skips the CSP pass."""
        ctx.bind_stream()
        n = atoms.n
        if n != self.n:
            raise ValueError("atom count differs from the state's")
        dev = atoms.pos.device
        f64 = dict(dtype=torch.float64, device=dev)
        out = dict(csp=csp if csp is not None else torch.empty(n, **f64), csp_avg=torch.empty(n, **f64),
                   w0=torch.empty(n, **f64), w_min=torch.empty(n, **f64), w_avg=torch.empty(n, **f64),
                   mask=torch.empty(n, dtype=torch.uint8, device=dev),
                   active=torch.empty(max(n, 1), dtype=torch.int32, device=dev))
        st = B.AvgState(self.n_avg, self.window, self.samples, self.dw_min, self.csp_ring.data_ptr(),
                        self.w_ring.data_ptr())
        na = C.c_int64(0)
        a, s, pp = atoms.struct(), nl.struct(), prec_struct(params, csp is not None)
        ctx._check(ctx.lib.apx_compute_precision_avg(ctx.h, C.byref(a), C.byref(s), C.byref(pp), C.byref(st),
                                                     _p(w0_extra), _p(out["csp"]), _p(out["csp_avg"]),
                                                     _p(out["w0"]), _p(out["w_min"]), _p(out["w_avg"]),
                                                     _p(self.w), _p(out["mask"]), _p(out["active"]), C.byref(na)))
        self.samples = int(st.samples)
        out["w"] = self.w.clone()
        out["n_active"] = int(na.value)
        out["active"] = out["active"][: out["n_active"]]
        return out


def eam_forces(ctx: Context, atoms: DeviceAtoms, nl: NeighborList, params, w=None) -> dict:
    ctx.bind_stream()
    n = atoms.n
    dev = atoms.pos.device
    out = dict(e_site=torch.empty(n, dtype=torch.float64, device=dev),
               rho=torch.empty(n, dtype=torch.float64, device=dev),
               f=torch.empty((3, n), dtype=torch.float64, device=dev))
    a, s, ep = atoms.struct(), nl.struct(), eam_struct(params)
    ctx._check(ctx.lib.apx_eam_forces(ctx.h, C.byref(a), C.byref(s), C.byref(ep), _p(w), _p(out["e_site"]),
                                      _p(out["rho"]), _p(out["f"])))
    return out


def num_basis(n_max: int, l_max: int) -> int:
    return int(B.load().apx_ace_num_basis(n_max, l_max))


class AceModel:
    """Device copy of an ACE parameter set (n_max, l_max, W, c1, c2, rc, h, s_a, eps, anchor)."""

    def __init__(self, ctx: Context, prm):
        self.ctx = ctx
        self.n_max, self.l_max = int(prm.n_max), int(prm.l_max)
        self.n_basis = num_basis(self.n_max, self.l_max)
        W = np.ascontiguousarray(prm.W, dtype=np.float64)
        c1 = np.ascontiguousarray(prm.c1, dtype=np.float64)
        c2 = np.ascontiguousarray(prm.c2, dtype=np.float64)
        if W.shape != (self.l_max + 1, self.n_max, self.n_max) or c1.size != self.n_basis or c2.size != self.n_basis:
            raise ValueError("ACE parameter shapes do not match the basis")
        d = B.AceDesc()
        d.n_max, d.l_max = self.n_max, self.l_max
        d.r_cut = float(getattr(prm, "rc", 5.0))
        d.h = float(getattr(prm, "h", 0.5))
        d.s_a = float(getattr(prm, "s_a", 1.0))
        d.eps = float(getattr(prm, "eps", 0.1))
        d.W, d.c1, d.c2 = W.ctypes.data, c1.ctypes.data, c2.ctypes.data
        anchor = getattr(prm, "anchor", None)
        d.anchored = 1 if anchor is not None else 0
        if anchor is not None:
            d.anchor = eam_struct(anchor)
        self._keep = (W, c1, c2)
        h = C.c_void_p()
        ctx._check(ctx.lib.apx_ace_model_create(ctx.h, C.byref(d), C.byref(h)))
        self.h = h

    def set_coeffs(self, c1, c2):
        """Replaces c1, c2 (host float64 arrays of length n_basis)."""
        c1 = np.ascontiguousarray(c1, dtype=np.float64)
        c2 = np.ascontiguousarray(c2, dtype=np.float64)
        if c1.size != self.n_basis or c2.size != self.n_basis:
            raise ValueError("coefficient vectors must have n_basis entries")
        self.ctx.bind_stream()
        self.ctx._check(self.ctx.lib.apx_ace_model_set_coeffs(self.ctx.h, self.h, c1.ctypes.data, c2.ctypes.data))

    def stats(self) -> dict:
        """Per-atom work counts of the coupling tables."""
        arr = (C.c_int64 * 6)()
        self.ctx._check(self.ctx.lib.apx_ace_model_stats(self.h, arr))
        keys = ("pairs", "triples", "coupling_terms", "triple_width", "n_basis", "n_atomic_base")
        return dict(zip(keys, (int(v) for v in arr)))

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.apx_ace_model_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ace_energy_forces(ctx: Context, atoms: DeviceAtoms, nl: NeighborList, model: AceModel,
                      active: torch.Tensor, w=None, precision: str = "fp64", want_dc: bool = False) -> dict:
    ctx.bind_stream()
    n = atoms.n
    dev = atoms.pos.device
    out = dict(e_site=torch.empty(n, dtype=torch.float64, device=dev),
               f=torch.empty((3, n), dtype=torch.float64, device=dev))
    dc1 = dc2 = None
    if want_dc:
        dc1 = torch.empty(model.n_basis, dtype=torch.float64, device=dev)
        dc2 = torch.empty(model.n_basis, dtype=torch.float64, device=dev)
    active = active.to(torch.int32).contiguous()
    prec = B.APX_FP32 if precision == "fp32" else B.APX_FP64
    a, s = atoms.struct(), nl.struct()
    ctx._check(ctx.lib.apx_ace_energy_forces(ctx.h, C.byref(a), C.byref(s), model.h, _p(w), _p(active),
                                             int(active.numel()), prec, _p(out["e_site"]), _p(out["f"]),
                                             _p(dc1), _p(dc2)))
    if want_dc:
        out["dE_dc1"], out["dE_dc2"] = dc1, dc2
    return out


def blend(ctx: Context, w, e_eam, e_ace, f_eam, f_ace, out=None, noalloc: bool = False) -> dict:
    """apx_blend, or apx_blend_noalloc with ``noalloc``; ``out`` supplies the output tensors."""
    ctx.bind_stream()
    n = int(e_eam.numel())
    dev = e_eam.device
    if out is None:
        out = dict(e_site=torch.empty(n, dtype=torch.float64, device=dev),
                   f=torch.empty((3, n), dtype=torch.float64, device=dev),
                   e_pot=torch.empty(1, dtype=torch.float64, device=dev))
    fn = ctx.lib.apx_blend_noalloc if noalloc else ctx.lib.apx_blend
    ctx._check(fn(ctx.h, n, _p(w), _p(e_eam), _p(e_ace), _p(f_eam), _p(f_ace),
                  _p(out["e_site"]), _p(out["f"]), _p(out["e_pot"])))
    return out


class MD:
    """Device-resident velocity-Verlet integrator (apx_md_*)."""

    def __init__(self, ctx: Context, atoms: DeviceAtoms, eam, ace: AceModel | None, prec, *, dt=1e-3,
                 mass=63.546, skin=0.5, max_nb=80, precision_every=10, ace_precision="fp32",
                 mode="adaptive", indenter=None, avg_samples=0, avg_dw_min=0.0, avg_window="past",
                 thermostat=None):
        """``thermostat``: None, or dict(r_omega, omega_max, seed) for the local thermostat."""
        self.ctx = ctx
        self.atoms = atoms
        p = B.MdParams()
        p.avg_samples, p.avg_dw_min = int(avg_samples), float(avg_dw_min)
        p.avg_window = {"past": B.WINDOW_PAST, "current": B.WINDOW_CURRENT}[avg_window]
        if thermostat is not None:
            p.thermostat = 1
            p.thermo = thermo_struct(thermostat)
        p.dt, p.mass, p.skin, p.max_nb = float(dt), float(mass), float(skin), int(max_nb)
        p.precision_every = int(precision_every)
        p.ace_precision = B.APX_FP32 if ace_precision == "fp32" else B.APX_FP64
        p.mode = {"adaptive": B.MODE_ADAPTIVE, "full_ace": B.MODE_FULL_ACE, "eam": B.MODE_EAM}[mode]
        if indenter is not None:
            p.indenter = 1
            p.ind_radius = float(indenter["radius"])
            p.ind_k = float(indenter["k"])
            for d in range(3):
                p.ind_center[d] = float(indenter["center"][d])
                p.ind_velocity[d] = float(indenter["velocity"][d])
        self._params = p
        self._eam = eam_struct(eam)
        self._prec = prec_struct(prec) if prec is not None else None
        a = atoms.struct()
        h = C.c_void_p()
        ctx.bind_stream()
        ctx._check(ctx.lib.apx_md_create(ctx.h, C.byref(a), C.byref(p), C.byref(self._eam),
                                         ace.h if ace is not None else None,
                                         C.byref(self._prec) if self._prec is not None else None, C.byref(h)))
        self.h = h
        self.ace = ace

    def init(self, pos: torch.Tensor):
        self.ctx.bind_stream()
        n = pos.shape[1]
        f = torch.empty((3, n), dtype=torch.float64, device=pos.device)
        w = torch.empty(n, dtype=torch.float64, device=pos.device)
        self.ctx._check(self.ctx.lib.apx_md_init(self.h, _p(pos), _p(f), _p(w)))
        return f, w

    def step(self, pos, vel, f, w, n_steps: int, allow_radicand: bool = False) -> dict:
        """apx_verlet_step; with ``allow_radicand`` a skipped thermostat correction returns
        the stats (key ``status``) instead of raising."""
        self.ctx.bind_stream()
        st = B.MdStats()
        code = self.ctx.lib.apx_verlet_step(self.h, _p(pos), _p(vel), _p(f), _p(w), int(n_steps), C.byref(st))
        if not (allow_radicand and code == B.APX_ERADICAND):
            self.ctx._check(code)
        out = {k: getattr(st, k) for k, _ in B.MdStats._fields_}
        out["status"] = int(code)
        return out

    def set_mlp(self, net, tau_lo: float, tau_hi: float):
        """Learned criterion (None: centro-symmetry alone)."""
        self.net = net
        self.ctx._check(self.ctx.lib.apx_md_set_mlp(self.h, net.h if net is not None else None, float(tau_lo),
                                                    float(tau_hi)))

    def timings(self) -> list:
        arr = (C.c_double * 5)()
        self.ctx._check(self.ctx.lib.apx_md_timings(self.h, arr))
        return list(arr)

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.apx_md_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_labels(ctx: Context, f_precise, f_fast):
    """apx_mlp_labels: (dF float64 [n], label float32 [n])."""
    ctx.bind_stream()
    n = int(f_precise.shape[1])
    dF = torch.empty(n, dtype=torch.float64, device=f_precise.device)
    label = torch.empty(n, dtype=torch.float32, device=f_precise.device)
    ctx._check(ctx.lib.apx_mlp_labels(ctx.h, n, _p(f_precise), _p(f_fast), _p(dF), _p(label)))
    return dF, label


def feature_stats(ctx: Context, feat) -> dict:
    """apx_mlp_feature_stats: per-column mean, sd (n - 1), min and max (host float64 [4] each)."""
    ctx.bind_stream()
    out = torch.empty(16, dtype=torch.float64, device=feat.device)
    ctx._check(ctx.lib.apx_mlp_feature_stats(ctx.h, _p(feat), int(feat.shape[0]), _p(out)))
    v = out.cpu().numpy()
    return dict(mean=v[0:4], sd=v[4:8], min=v[8:12], max=v[12:16])


def weighted_sum(ctx: Context, w, e) -> torch.Tensor:
    """apx_weighted_sum: 0-d tensor sum_i w_i e_i (w None: all 1)."""
    ctx.bind_stream()
    out = torch.empty((), dtype=torch.float64, device=e.device)
    ctx._check(ctx.lib.apx_weighted_sum(ctx.h, int(e.numel()), _p(w), _p(e), _p(out)))
    return out


def thermo_struct(p) -> B.ThermoParams:
    t = B.ThermoParams()
    t.r_omega = float(p["r_omega"])
    t.omega_max = int(p["omega_max"])
    t.group_batch = int(p.get("group_batch", 0))
    t.seed = int(p["seed"])
    return t


def thermostat_energy_errors(ctx: Context, w_c, w_d, e_fast, e_precise, f_d, df, v_half, dt: float, mass: float,
                             frozen=None) -> torch.Tensor:
    """apx_thermostat_energy_errors: dE [n]."""
    ctx.bind_stream()
    n = int(w_c.numel())
    dE = torch.empty(n, dtype=torch.float64, device=w_c.device)
    ctx._check(ctx.lib.apx_thermostat_energy_errors(ctx.h, n, _p(frozen), _p(w_c), _p(w_d), _p(e_fast),
                                                    _p(e_precise), _p(f_d), _p(df), _p(v_half), float(dt),
                                                    float(mass), _p(dE)))
    return dE


def thermostat_correct(ctx: Context, atoms: DeviceAtoms, vel, dE, params, step: int, mass: float,
                       allow_radicand: bool = False) -> dict:
    """apx_thermostat_correct on ``vel`` (in place): dict(corrected, failed, status)."""
    ctx.bind_stream()
    a = atoms.struct()
    tp = thermo_struct(params)
    nc, nf = C.c_int64(0), C.c_int64(0)
    code = ctx.lib.apx_thermostat_correct(ctx.h, C.byref(a), _p(vel), _p(dE), C.byref(tp), int(step), float(mass),
                                          C.byref(nc), C.byref(nf))
    if not (allow_radicand and code == B.APX_ERADICAND):
        ctx._check(code)
    return dict(corrected=int(nc.value), failed=int(nf.value), status=int(code))


def features(ctx: Context, atoms: DeviceAtoms, nl: NeighborList, rho, csp, f_eam) -> torch.Tensor:
    """[n, 4] float32 features of the learned criterion."""
    ctx.bind_stream()
    feat = torch.empty((atoms.n, 4), dtype=torch.float32, device=atoms.pos.device)
    a, s = atoms.struct(), nl.struct()
    ctx._check(ctx.lib.apx_features(ctx.h, C.byref(a), C.byref(s), _p(rho), _p(csp), _p(f_eam), _p(feat)))
    return feat


class Mlp:
    """Device copy of the learned criterion's network (apx_mlp_*)."""

    N_PARAMS = B.MLP_PARAMS

    def __init__(self, ctx: Context, params, mu, sd):
        self.ctx = ctx
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.N_PARAMS:
            raise ValueError("wrong parameter count")
        mu = np.ascontiguousarray(mu, dtype=np.float32)
        sd = np.ascontiguousarray(sd, dtype=np.float32)
        h = C.c_void_p()
        ctx._check(ctx.lib.apx_mlp_create(ctx.h, p.ctypes.data, mu.ctypes.data, sd.ctypes.data, C.byref(h)))
        self.h = h
        self.loss = torch.zeros(1, dtype=torch.float32, device=ctx.torch_device)

    def params(self) -> np.ndarray:
        out = np.empty(self.N_PARAMS, dtype=np.float32)
        self.ctx.bind_stream()
        self.ctx._check(self.ctx.lib.apx_mlp_get_params(self.ctx.h, self.h, out.ctypes.data))
        return out

    def set_range(self, fmin, fmax):
        a = np.ascontiguousarray(fmin, dtype=np.float32)
        b = np.ascontiguousarray(fmax, dtype=np.float32)
        self.ctx._check(self.ctx.lib.apx_mlp_set_range(self.h, a.ctypes.data, b.ctypes.data))

    def forward(self, feat: torch.Tensor) -> torch.Tensor:
        self.ctx.bind_stream()
        out = torch.empty(feat.shape[0], dtype=torch.float32, device=feat.device)
        self.ctx._check(self.ctx.lib.apx_mlp_forward(self.ctx.h, self.h, _p(feat), feat.shape[0], _p(out)))
        return out

    def gradients(self, feat, target, sel=None):
        self.ctx.bind_stream()
        g = torch.empty(self.N_PARAMS, dtype=torch.float32, device=feat.device)
        nb = int(sel.numel()) if sel is not None else int(feat.shape[0])
        self.ctx._check(self.ctx.lib.apx_mlp_gradients(self.ctx.h, self.h, _p(feat), _p(target), _p(sel), nb,
                                                       _p(g), _p(self.loss)))
        return g, self.loss

    def adam_step(self, grad, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.ctx.bind_stream()
        self.ctx._check(self.ctx.lib.apx_mlp_adam_step(self.ctx.h, self.h, _p(grad), lr, b1, b2, eps))

    def train_step(self, feat, target, sel, lr=1e-3):
        self.ctx.bind_stream()
        self.ctx._check(self.ctx.lib.apx_mlp_train_step(self.ctx.h, self.h, _p(feat), _p(target), _p(sel),
                                                        int(sel.numel()), lr, _p(self.loss)))
        return self.loss

    def infer_bf16(self, feat: torch.Tensor) -> torch.Tensor:
        self.ctx.bind_stream()
        out = torch.empty(feat.shape[0], dtype=torch.float32, device=feat.device)
        self.ctx._check(self.ctx.lib.apx_mlp_infer_bf16(self.ctx.h, self.h, _p(feat), feat.shape[0], _p(out)))
        return out

    def weight(self, pred: torch.Tensor, feat: torch.Tensor, tau_lo: float, tau_hi: float) -> torch.Tensor:
        """apx_mlp_weight: the learned detection weight of given predictions."""
        self.ctx.bind_stream()
        n = int(pred.numel())
        w0 = torch.empty(n, dtype=torch.float64, device=pred.device)
        self.ctx._check(self.ctx.lib.apx_mlp_weight(self.ctx.h, self.h, _p(pred), _p(feat), n, float(tau_lo),
                                                    float(tau_hi), _p(w0)))
        return w0

    def precision(self, feat: torch.Tensor, tau_lo: float, tau_hi: float):
        self.ctx.bind_stream()
        n = feat.shape[0]
        pred = torch.empty(n, dtype=torch.float32, device=feat.device)
        w0 = torch.empty(n, dtype=torch.float64, device=feat.device)
        self.ctx._check(self.ctx.lib.apx_mlp_precision(self.ctx.h, self.h, _p(feat), n, float(tau_lo), float(tau_hi),
                                                       _p(pred), _p(w0)))
        return pred, w0

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.apx_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
