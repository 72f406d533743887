"""Python binding of the QSA library: argument marshalling around libqsa.so.

torch provides the device workspace and the stream; every step of the slice
sweep and the beam push runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional, Sequence

import numpy as np
import torch

from . import _lib as L

_PREC = {"f64": L.QSA_FP64, "fp64": L.QSA_FP64, "f32": L.QSA_FP32, "fp32": L.QSA_FP32}


def _ptr(a) -> int:
    return a.data_ptr() if isinstance(a, torch.Tensor) else a.ctypes.data


def _f64(a):
    """A float64 contiguous host array or device tensor (on_device flag)."""
    if isinstance(a, torch.Tensor):
        if a.is_cuda:
            return a.to(torch.float64).contiguous(), 1
        return np.ascontiguousarray(a.numpy(), dtype=np.float64), 0
    return np.ascontiguousarray(a, dtype=np.float64), 0


def make_params(nx: int, ny: int, nxi: int, dx: float, dy: float, dxi: float, dt: float,
                species: Sequence, n_plasma: int, plasma_w: float,
                beam_capacity: Sequence[int], precision: str = "f64", n_corr: int = 3,
                kappa2: float = 0.75, pipeline: int = 1, adjoint_steps: int = 0,
                ckpt_every: int = 0, field_pack: bool = True,
                plasma_weights: bool = False, lean_pipeline: bool = False,
                b0z: float = 0.0, ion_m: float = 0.0, ion_z: int = 1) -> L.QSAParams:
    """species: sequence of (Z, M); pipeline: beam steps in flight (1 = off);
    adjoint_steps: most steps qsa_adjoint_sweep differentiates (0 = none);
    ckpt_every: the adjoint's plasma checkpoint stride in slices (0 = 16);
    field_pack: keep the push's fields packed for every slice (without steps
    in flight; False saves 32-48 bytes per cell); plasma_weights: keep a
    weight per plasma macro-particle (Sim.load_plasma loads them when the
    template's "w" is an array); lean_pipeline: steps in flight without a
    second copy of the beam (read_beam then returns storage order); b0z: a
    uniform external magnetic field along the propagation axis; ion_m, ion_z:
    mass (in m_e; 0 = immobile ions) and charge number of mobile plasma ions."""
    p = L.QSAParams()
    p.nx, p.ny, p.nxi = nx, ny, nxi
    p.precision = _PREC[precision]
    p.dx, p.dy, p.dxi, p.dt = dx, dy, dxi, dt
    p.n_corr, p.kappa2 = n_corr, kappa2
    p.n_plasma, p.plasma_w = n_plasma, plasma_w
    p.n_species = len(species)
    p.pipeline = int(pipeline)
    p.adjoint_steps = int(adjoint_steps)
    p.ckpt_every = int(ckpt_every)
    p.no_field_pack = 0 if field_pack else 1
    p.plasma_weights = 1 if plasma_weights else 0
    p.lean_pipeline = 1 if lean_pipeline else 0
    p.b0z = float(b0z)
    p.ion_m = float(ion_m)
    p.ion_z = int(ion_z)
    for i, (Z, M) in enumerate(species):
        p.species[i].Z = int(Z)
        p.species[i].M = float(M)
        p.beam_capacity[i] = int(beam_capacity[i])
    return p


def params_from_workload(wl, precision: Optional[str] = None,
                         beam_capacity: Optional[Sequence[int]] = None,
                         pipeline: int = 1, adjoint_steps: int = 0,
                         ckpt_every: Optional[int] = None, field_pack: bool = True,
                         lean_pipeline: bool = False) -> L.QSAParams:
    """Parameters of a workload description (duck-typed: grid, species, loading)."""
    caps = beam_capacity or [wl.n_beam(s) for s in range(len(wl.species))]
    ck = getattr(wl, "ckpt_every", 0) if ckpt_every is None else ckpt_every
    return make_params(wl.nx, wl.ny, wl.nxi, wl.dx, wl.dy, wl.dxi, wl.dt,
                       [(s.Z, s.M) for s in wl.species], wl.n_plasma,
                       wl.dx * wl.dy / wl.plasma_ppc, caps, precision or wl.precision,
                       wl.n_corr, wl.kappa2, pipeline, adjoint_steps, min(int(ck), wl.nxi), field_pack,
                       (getattr(wl, "plasma_w_spread", 0.0) > 0.0 or getattr(wl, "plasma_n0", 1.0) != 1.0
                        or getattr(wl, "plasma_mod", 0.0) != 0.0 or getattr(wl, "ion_m", 0.0) > 0.0),
                       lean_pipeline, float(getattr(wl, "b0z", 0.0)), float(getattr(wl, "ion_m", 0.0)),
                       int(getattr(wl, "ion_z", 1)))


class Sim:
    """One simulation box on the current CUDA (HIP) device."""

    def __init__(self, params: L.QSAParams, device: str = "cuda",
                 stream: Optional[torch.cuda.Stream] = None):
        self.lib = L.lib()
        self.params = params
        nbytes = self.lib.qsa_workspace_bytes(C.byref(params))
        if nbytes == 0:
            raise L.QSAError(-1, "invalid parameters")
        self.device = torch.device(device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        # 256-byte aligned workspace owned by the caller (torch)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws = (base + 255) // 256 * 256
        self.ws_bytes = nbytes
        ctx = C.c_void_p()
        self._check(self.lib.qsa_create(C.byref(params), C.c_void_p(self._ws), nbytes,
                                        C.c_void_p(self.stream.cuda_stream), C.byref(ctx)), None)
        self.ctx = ctx
        self.nperp = params.nx * params.ny

    # ------------------------------------------------------------------
    def _check(self, st: int, ctx=-1):
        if st != L.QSA_OK:
            c = self.ctx if ctx == -1 else ctx
            msg = self.lib.qsa_last_error(c).decode() if c else L.STATUS.get(st, "")
            raise L.QSAError(st, msg)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.qsa_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def load_plasma(self, plasma: Dict):
        """The plasma template; a "w" array (one weight per particle, in the
        units of plasma_w) needs a context made with plasma_weights."""
        arrs = [_f64(plasma[k]) for k in ("x", "y", "ux", "uy")]
        n = arrs[0][0].shape[0]
        on_dev = arrs[0][1]
        w = plasma.get("w")
        per_particle = w is not None and (w.dim() > 0 if torch.is_tensor(w) else np.ndim(w) > 0)
        if per_particle and not self.params.plasma_weights:
            raise ValueError("per-particle plasma weights need a context made with plasma_weights")
        self._check(self.lib.qsa_load_plasma(self.ctx, *[C.c_void_p(_ptr(a)) for a, _ in arrs],
                                             n, on_dev))
        kind = plasma.get("kind")
        if kind is not None:
            # the library marks a mobile ion (kind 1) by a negative weight
            if torch.is_tensor(w) or torch.is_tensor(kind):
                kt = torch.as_tensor(kind)
                wt = torch.as_tensor(w, dtype=torch.float64, device=kt.device).expand(kt.shape)
                w = torch.where(kt > 0, -wt, wt)
            else:
                sign = np.where(np.asarray(kind) > 0, -1.0, 1.0)
                w = sign * np.broadcast_to(np.asarray(w, dtype=np.float64), sign.shape)
            per_particle = True
        if per_particle:
            wa, wdev = _f64(w)
            self._check(self.lib.qsa_load_plasma_weights(self.ctx, C.c_void_p(_ptr(wa)), wa.shape[0], wdev))
        ion = plasma.get("ion")
        if ion is not None:
            self.load_ions(ion)

    def load_ions(self, ion):
        """The immobile ions' density at the nodes, [ny, nx] (a context made
        with plasma_weights)."""
        if not self.params.plasma_weights:
            raise ValueError("an ion density profile needs a context made with plasma_weights")
        ia, idev = _f64(ion)
        ia = ia.reshape(-1)
        self._check(self.lib.qsa_load_ions(self.ctx, C.c_void_p(_ptr(ia)), ia.shape[0], idev))

    def load_beam(self, s: int, beam: Dict):
        arrs = [_f64(beam[k]) for k in ("x", "y", "xi", "ux", "uy", "uz", "w")]
        n = arrs[0][0].shape[0]
        on_dev = arrs[0][1]
        self._check(self.lib.qsa_load_beam(self.ctx, s, *[C.c_void_p(_ptr(a)) for a, _ in arrs],
                                           n, on_dev))

    def load_beam_range(self, s: int, first: int, beam: Dict):
        """Particles [first, first + n) of species s (first = 0 starts a new
        beam, first = the current count appends)."""
        arrs = [_f64(beam[k]) for k in ("x", "y", "xi", "ux", "uy", "uz", "w")]
        n = arrs[0][0].shape[0]
        on_dev = arrs[0][1]
        self._check(self.lib.qsa_load_beam_range(self.ctx, s, int(first),
                                                 *[C.c_void_p(_ptr(a)) for a, _ in arrs], n, on_dev))

    def read_beam(self, s: int) -> Dict[str, np.ndarray]:
        cap = int(self.params.beam_capacity[s])
        out = {k: np.empty(cap) for k in ("x", "y", "xi", "ux", "uy", "uz", "w")}
        n = C.c_int64()
        self._check(self.lib.qsa_read_beam(
            self.ctx, s, *[C.c_void_p(out[k].ctypes.data) for k in ("x", "y", "xi", "ux", "uy", "uz", "w")],
            cap, C.byref(n), 0))
        return {k: v[:n.value] for k, v in out.items()}

    def slice_sweep(self):
        self._check(self.lib.qsa_slice_sweep(self.ctx))

    def beam_step(self, n: int = 1):
        self._check(self.lib.qsa_beam_step(self.ctx, n))

    def sync(self):
        self._check(self.lib.qsa_sync(self.ctx))

    def set_graphs(self, enable: bool):
        """Replay captured HIP graphs (default) or enqueue every launch."""
        self._check(self.lib.qsa_set_option(self.ctx, 0, int(bool(enable))))

    def set_pipeline(self, depth: int):
        """Beam steps in flight (1 .. the pipeline parameter)."""
        self._check(self.lib.qsa_set_option(self.ctx, 1, int(depth)))

    def set_beam_beside(self, enable: bool):
        """One step at a time: run the beam deposit and push beside the slice
        loop on a second stream (default) or after it."""
        self._check(self.lib.qsa_set_option(self.ctx, 5, int(bool(enable))))

    def set_beside_blocks(self, n: int):
        """Workgroups per launch of the beam work beside the slice loop (0 =
        as many as the work has)."""
        self._check(self.lib.qsa_set_option(self.ctx, 6, int(n)))

    def set_resort_every(self, n: int):
        """One step at a time: reorder the beam storage by deposit key before
        every n-th beam step (0 = never); read_beam then returns particles in
        storage order."""
        self._check(self.lib.qsa_set_option(self.ctx, 7, int(n)))

    def set_shapes(self, plasma_threads: int = 0, row_threads: int = 0, col_threads: int = 0):
        """Launch shapes (0 = default): threads per plasma-row block, per
        row-transform block and per column transform."""
        self._check(self.lib.qsa_set_option(self.ctx, 2, int(plasma_threads)))
        self._check(self.lib.qsa_set_option(self.ctx, 3, int(row_threads)))
        self._check(self.lib.qsa_set_option(self.ctx, 4, int(col_threads)))

    def shapes(self):
        """(threads per plasma-row block, per row-transform block, per column
        transform) in use."""
        out = []
        for opt in (2, 3, 4):
            v = C.c_int64(0)
            self._check(self.lib.qsa_get_option(self.ctx, opt, C.byref(v)))
            out.append(int(v.value))
        return tuple(out)

    def adjoint_sweep(self, n_steps: int, amps, bins):
        """Transverse magnetic energy after n_steps beam steps with the weights
        scaled by amps[bin] and its gradient with respect to amps.  bins: one
        int array per species in load order.  Returns (loss, grad ndarray)."""
        amps = np.ascontiguousarray(np.asarray(amps, dtype=np.float64))
        arrs = [np.ascontiguousarray(np.asarray(b, dtype=np.int32)) for b in bins]
        ptrs = (C.POINTER(C.c_int32) * len(arrs))(
            *[a.ctypes.data_as(C.POINTER(C.c_int32)) for a in arrs])
        loss = C.c_double(0.0)
        grad = np.zeros(amps.size, dtype=np.float64)
        self._check(self.lib.qsa_adjoint_sweep(
            self.ctx, int(n_steps), int(amps.size), amps.ctypes.data_as(C.POINTER(C.c_double)), ptrs,
            C.byref(loss), grad.ctypes.data_as(C.POINTER(C.c_double))))
        return float(loss.value), grad

    def autotune(self) -> float:
        """Time the launch shapes and steps in flight on this machine's data and
        keep the fastest; returns the best ms per step (per sweep without
        pipelining)."""
        ms = C.c_double(0.0)
        self._check(self.lib.qsa_autotune(self.ctx, C.byref(ms)))
        return float(ms.value)

    @property
    def pipeline(self) -> int:
        """Beam steps in flight in use (1 after a drift fallback)."""
        v = C.c_int64(0)
        self._check(self.lib.qsa_get_option(self.ctx, 1, C.byref(v)))
        return int(v.value)

    def timing_begin(self, kernel_class: str):
        """Time every launch of one kernel class with HIP events on the stream."""
        self._check(self.lib.qsa_timing_begin(self.ctx, L.KERNEL_CLASSES[kernel_class]))

    def timing_end(self):
        """-> (summed kernel milliseconds, number of timed launches)."""
        ms = C.c_double()
        n = C.c_int64()
        self._check(self.lib.qsa_timing_end(self.ctx, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def fields(self, name: str, xi0: int = 0, xi1: Optional[int] = None,
               on_device: bool = False):
        """Slices [xi0, xi1) of one field as float64 [nxi, ny, nx] (numpy, or a
        device tensor with on_device)."""
        p = self.params
        xi1 = p.nxi if xi1 is None else xi1
        shape = (xi1 - xi0, p.ny, p.nx)
        n = int(np.prod(shape))
        if on_device:
            out = torch.empty(shape, dtype=torch.float64, device=self.device)
            self._check(self.lib.qsa_fields(self.ctx, L.FIELD_IDS[name], xi0, xi1,
                                            C.c_void_p(out.data_ptr()), n, 1))
        else:
            out = np.empty(shape)
            self._check(self.lib.qsa_fields(self.ctx, L.FIELD_IDS[name], xi0, xi1,
                                            C.c_void_p(out.ctypes.data), n, 0))
        return out

    FIELD_MOMENTS = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")
    BEAM_MOMENTS = ("w", "wux", "wuy", "wuz", "wux2", "wuy2", "wuz2")

    def field_moments(self, window: int = 1, on_device: bool = False):
        """[n_windows, 6] float64: per window of `window` slices, the mean of
        the transverse means of E_x^2, E_y^2, E_z^2, B_x^2, B_y^2, B_z^2 of
        the last sweep (qsa_field_moments)."""
        nw = -(-self.params.nxi // window) if window >= 1 else 1   # the library rejects window < 1
        if on_device:
            out = torch.empty((nw, 6), dtype=torch.float64, device=self.device)
            self._check(self.lib.qsa_field_moments(self.ctx, window, C.c_void_p(out.data_ptr()), out.numel(), 1))
        else:
            out = np.empty((nw, 6))
            self._check(self.lib.qsa_field_moments(self.ctx, window, C.c_void_p(out.ctypes.data), out.size, 0))
        return out

    def beam_moments(self, species: int = 0, window: int = 1, on_device: bool = False):
        """[n_windows, 7] float64: per window of `window` slices, the sums of
        (w, w u_x, w u_y, w u_z, w u_x^2, w u_y^2, w u_z^2) over the beam
        particles of species s in it (qsa_beam_moments)."""
        nw = -(-self.params.nxi // window) if window >= 1 else 1
        if on_device:
            out = torch.empty((nw, 7), dtype=torch.float64, device=self.device)
            self._check(self.lib.qsa_beam_moments(self.ctx, species, window, C.c_void_p(out.data_ptr()),
                                                  out.numel(), 1))
        else:
            out = np.empty((nw, 7))
            self._check(self.lib.qsa_beam_moments(self.ctx, species, window, C.c_void_p(out.ctypes.data),
                                                  out.size, 0))
        return out


class Batch:
    """Several Sims advanced together: their slice loops run as lanes of the
    same kernel launches (one launch per phase per slice for the batch)."""

    def __init__(self, sims: Sequence[Sim], stream: Optional[torch.cuda.Stream] = None):
        if not sims:
            raise ValueError("empty batch")
        self.lib = L.lib()
        self.sims = list(sims)
        n = len(self.sims)
        nbytes = self.lib.qsa_batch_workspace_bytes(n)
        dev = self.sims[0].device
        self.stream = stream or torch.cuda.current_stream(dev)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        ws = (self.workspace.data_ptr() + 255) // 256 * 256
        arr = (C.c_void_p * n)(*[s.ctx.value for s in self.sims])
        b = C.c_void_p()
        st = self.lib.qsa_batch_create(arr, n, C.c_void_p(ws), nbytes,
                                       C.c_void_p(self.stream.cuda_stream), C.byref(b))
        if st != L.QSA_OK:
            raise L.QSAError(st, "qsa_batch_create failed")
        self.b = b

    def _check(self, st):
        if st != L.QSA_OK:
            msg = self.lib.qsa_last_error(self.sims[0].ctx).decode()
            raise L.QSAError(st, msg)

    def sweep(self):
        self._check(self.lib.qsa_batch_sweep(self.b))

    def step(self, n: int = 1):
        self._check(self.lib.qsa_batch_step(self.b, n))

    def sync(self):
        self._check(self.lib.qsa_batch_sync(self.b))

    def close(self):
        if getattr(self, "b", None):
            self.lib.qsa_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_sweep_static(sims: Sequence[Sim], stream: Optional[torch.cuda.Stream] = None):
    """One sweep of every Sim as lanes of the same launches, with the lane
    table in the library's static device memory (qsa_batch_sweep_static: no
    batch object, no workspace, nothing allocated).  `stream` defaults to
    the first Sim's stream."""
    if not sims:
        raise ValueError("empty batch")
    lib = L.lib()
    st = stream if stream is not None else sims[0].stream
    arr = (C.c_void_p * len(sims))(*[s.ctx.value for s in sims])
    status = lib.qsa_batch_sweep_static(arr, len(sims), C.c_void_p(st.cuda_stream))
    if status != L.QSA_OK:
        raise L.QSAError(status, lib.qsa_last_error(sims[0].ctx).decode())


def linear_model(gamma, n0, dxi: float, taus, dtau: float, device=None):
    """Batched solve of the single-mode linear model, Eq. (5)
    (qsa_linear_model): gamma [n_inst] growth rates, or [n_inst, nxi]
    longitudinal profiles Gamma(xi_j); n0 [n_inst, nxi] (or [nxi], shared)
    seeds on xi_j = j dxi; returns device tensors n and dPsi
    [n_inst, len(taus), nxi] at the output times taus (multiples of dtau
    from 0)."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    ga = np.asarray(gamma, dtype=np.float64)
    per_point = 1 if ga.ndim == 2 else 0
    if ga.ndim > 2:
        raise ValueError("gamma is [n_inst] or [n_inst, nxi]")
    g = torch.as_tensor(np.ascontiguousarray(ga if per_point else ga.reshape(-1))).to(dev)
    s0 = torch.as_tensor(np.asarray(n0, dtype=np.float64)).to(dev)
    if s0.dim() == 1:
        s0 = s0.expand(g.shape[0], -1)
    s0 = s0.contiguous()
    n_inst, nxi = s0.shape
    if g.shape[0] != n_inst or (per_point and g.shape[1] != nxi):
        raise ValueError("one gamma (or one profile of nxi points) per seed row")
    t = np.ascontiguousarray(np.asarray(taus, dtype=np.float64).reshape(-1))
    n_out = torch.empty((n_inst, t.size, nxi), dtype=torch.float64, device=dev)
    p_out = torch.empty_like(n_out)
    lib = L.lib()
    stream = torch.cuda.current_stream(dev).cuda_stream
    st = lib.qsa_linear_model(n_inst, nxi, float(dxi), float(dtau), C.c_void_p(g.data_ptr()), per_point,
                              C.c_void_p(s0.data_ptr()), t.size, t.ctypes.data_as(C.POINTER(C.c_double)),
                              C.c_void_p(n_out.data_ptr()), C.c_void_p(p_out.data_ptr()), C.c_void_p(stream))
    if st != L.QSA_OK:
        raise L.QSAError(st, "qsa_linear_model: arguments out of range or launch failed")
    return n_out, p_out


def dirichlet_solve(f: torch.Tensor, dx: float, dy: float, kappa2: float = 0.0,
                    out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Conducting-wall solve (qsa_dirichlet_solve) of (-lap_perp + kappa2) u = f
    on the interior nodes: f a device tensor [..., ny, nx] (float64 or
    float32; nx + 1 and ny + 1, unless ny = 1, powers of two); returns u of
    the same shape and dtype (out may be f)."""
    if not f.is_cuda or f.dtype not in (torch.float64, torch.float32) or f.dim() < 2:
        raise ValueError("f: a float64 or float32 device tensor [..., ny, nx]")
    f = f.contiguous()
    ny, nx = int(f.shape[-2]), int(f.shape[-1])
    n_grid = int(f.numel() // max(nx * ny, 1))
    u = torch.empty_like(f) if out is None else out
    if u.shape != f.shape or u.dtype != f.dtype or not u.is_contiguous():
        raise ValueError("out: a contiguous tensor of f's shape and dtype")
    prec = 0 if f.dtype == torch.float64 else 1
    stream = torch.cuda.current_stream(f.device).cuda_stream
    st = L.lib().qsa_dirichlet_solve(prec, n_grid, nx, ny, float(dx), float(dy), float(kappa2),
                                     C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()), C.c_void_p(stream))
    if st != L.QSA_OK:
        raise L.QSAError(st, "qsa_dirichlet_solve: arguments out of range or launch failed")
    return u


class FieldEnergy(torch.autograd.Function):
    """torch.autograd.Function over the library's adjoint: forward gives the
    transverse magnetic energy after n_steps beam steps as a function of the
    beam-amplitude bins, backward the library's reverse-mode gradient."""

    @staticmethod
    def forward(ctx, amps: torch.Tensor, sim: "Sim", n_steps: int, bins):
        loss, grad = sim.adjoint_sweep(n_steps, amps.detach().cpu().numpy(), bins)
        ctx.save_for_backward(torch.as_tensor(grad, dtype=amps.dtype))
        return torch.tensor(loss, dtype=amps.dtype)

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return g * grad, None, None, None
