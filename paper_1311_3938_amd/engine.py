"""Python front end of the HIP library: contexts, Hamiltonians, H|psi>,
time evolution and float64 reductions on torch device tensors.

torch provides the device memory and the stream; every computation is a call
into libaqc.so (include/aqc.h)."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from ._lib import check, lib


def dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.complex64:
        return L.C64
    if t.dtype == torch.complex128:
        return L.C128
    raise TypeError(f"state must be complex64 or complex128, got {t.dtype}")


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Context:
    """A device plus a HIP stream (torch's current stream by default)."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the engine runs on the HIP device only")
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        check(lib().aqc_create(device, C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def set_stream(self, stream: torch.cuda.Stream):
        self.stream = stream
        check(lib().aqc_set_stream(self._h, C.c_void_p(stream.cuda_stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().aqc_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def trim(device: int = 0):
    """Free the kept device buffers of released Hamiltonian tables (aqc_trim)."""
    check(lib().aqc_trim(int(device)))


class Hamiltonian:
    """Compiled form of an ``instances.Instance`` (terms, schedules, path)."""

    def __init__(self, ctx: Context, inst):
        self.ctx = ctx
        self.n = int(inst.n)
        x = np.ascontiguousarray(inst.x, dtype=np.uint64)
        z = np.ascontiguousarray(inst.z, dtype=np.uint64)
        w = np.ascontiguousarray(inst.w, dtype=np.float64)
        sid = np.ascontiguousarray(inst.sid, dtype=np.int32)
        ns = len(inst.scheds)
        sch = (L.Sched * ns)(*[L.make_sched(s) for s in inst.scheds])
        path = L.make_path(inst.path)
        h = C.c_void_p()
        u64p = C.POINTER(C.c_uint64)
        check(lib().aqc_build_hamiltonian(
            ctx.handle, self.n, len(w), x.ctypes.data_as(u64p), z.ctypes.data_as(u64p),
            w.ctypes.data_as(C.POINTER(C.c_double)), sid.ctypes.data_as(C.POINTER(C.c_int32)),
            ns, sch, C.byref(path), C.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    @property
    def dim(self):
        """Amplitudes of a state: 2^n (a sector: C(n, w))."""
        return int(lib().aqc_ham_dim(self._h))

    def info(self):
        i = L.HamInfo()
        check(lib().aqc_ham_info(self._h, C.byref(i)))
        return {"n_qubits": i.n_qubits, "n_terms": i.n_terms, "n_diag_terms": i.n_diag_terms,
                "n_groups": i.n_groups, "n_passes": list(i.n_passes),
                "tile_bits": list(i.tile_bits)}

    def set_tiling(self, dtype, tbf, tbh, lh, options=1):
        """options: register passes 0 none, 1 library's choice, 2 narrow, 3 wide
        (True = 1), plus 4 for stream groups in the last pass."""
        dt = L.C64 if dtype in (torch.complex64, L.C64) else L.C128
        check(lib().aqc_ham_set_tiling(self._h, dt, int(tbf), int(tbh), int(lh), int(options)))

    def spectral_bounds(self, t0, t1):
        lo, hi = C.c_double(), C.c_double()
        check(lib().aqc_spectral_bounds(self.ctx.handle, self._h, t0, t1, C.byref(lo), C.byref(hi)))
        return lo.value, hi.value

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().aqc_ham_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Sector(Hamiltonian):
    """A Hamiltonian that keeps the Hamming weight, restricted to the C(n, w)
    basis states of weight w (Sec. III.A.2-3), stored by increasing z.
    apply, evolve, energy, ground_mass and spectral_bounds take it like a
    Hamiltonian, on states of C(n, w) amplitudes."""

    def __init__(self, ctx: Context, ham: Hamiltonian, weight: int):
        self.ctx = ctx
        self.n = ham.n
        self.weight = int(weight)
        h = C.c_void_p()
        check(lib().aqc_sector_create(ctx.handle, ham.handle, self.weight, C.byref(h)))
        self._h = h

    def dicke(self, dtype=torch.complex64):
        """eq. (initstate): every amplitude of the sector C(n, w)^{-1/2}."""
        psi = torch.empty(self.dim, dtype=dtype, device=self.ctx.device)
        check(lib().aqc_sector_dicke(self.ctx.handle, self._h, _ptr(psi), dtype_code(psi)))
        return psi

    def expand(self, psi):
        """The 2^n state with the sector's amplitudes and zeros elsewhere."""
        _check_state(self.ctx, self, psi)
        out = torch.empty(1 << self.n, dtype=psi.dtype, device=psi.device)
        check(lib().aqc_sector_expand(self.ctx.handle, self._h, _ptr(psi), _ptr(out), dtype_code(psi)))
        return out


def _check_state(ctx, ham, psi):
    if psi.device != ctx.device:
        raise ValueError("state is not on the context's device")
    if not psi.is_contiguous():
        raise ValueError("state must be contiguous")
    if psi.numel() != ham.dim:
        raise ValueError(f"state has {psi.numel()} amplitudes, expected {ham.dim}")
    return dtype_code(psi)


def workspace(ctx, nbytes):
    if nbytes == 0:
        return None
    return torch.empty(nbytes, dtype=torch.uint8, device=ctx.device)


def apply(ctx: Context, ham: Hamiltonian, t: float, psi: torch.Tensor, out=None, ws=None):
    """out = H(t) psi."""
    dt = _check_state(ctx, ham, psi)
    if out is None:
        out = torch.empty_like(psi)
    need = lib().aqc_apply_workspace_bytes(ham.handle, dt)
    if need and ws is None:
        ws = workspace(ctx, need)
    check(lib().aqc_apply(ctx.handle, ham.handle, float(t), _ptr(psi), _ptr(out), dt,
                          _ptr(ws) if ws is not None else None, ws.numel() if ws is not None else 0))
    return out


def evolve_opts(method="pc4", n_steps=1000, shift=0.0, check_every=0, norm_tol=1e-3,
                stab_limit=0.0, atol=1e-9, h0=0.0, hmin=0.0, hmax=0.0, window=8, replay=None,
                record_cap=0, compensated=True):
    o = L.EvolveOpts()
    o.method = {"pc4": L.METHOD_PC4, "rk4": L.METHOD_RK4}[method]
    o.n_steps = int(n_steps)
    if isinstance(shift, str):
        if shift != "center":
            raise ValueError(shift)
        o.shift_mode = L.SHIFT_CENTER
    else:
        o.shift_mode = L.SHIFT_VALUE
        o.shift = float(shift)
    o.check_every = int(check_every)
    o.norm_tol = float(norm_tol)
    o.stab_limit = float(stab_limit)
    o.atol, o.h0, o.hmin, o.hmax = float(atol), float(h0), float(hmin), float(hmax)
    o.window = int(window)
    o.compensated = 1 if compensated else 0
    keep = []
    if replay is not None:
        arr = np.ascontiguousarray(np.asarray(replay, dtype=np.float64).reshape(-1, 3))
        keep.append(arr)
        o.n_replay = arr.shape[0]
        o.replay = arr.ctypes.data_as(C.POINTER(C.c_double))
    rec = None
    if record_cap:
        rec = np.zeros((record_cap, 3), dtype=np.float64)
        keep.append(rec)
        o.record = rec.ctypes.data_as(C.POINTER(C.c_double))
        o.record_cap = record_cap
    return o, keep, rec


def evolve_workspace_bytes(ham, dtype, opts):
    return lib().aqc_evolve_workspace_bytes(ham.handle, dtype, C.byref(opts))


def new_carry():
    """A fresh chain for consecutive fixed-step pc4 calls (aqc_pc4_carry)."""
    return L.Pc4Carry()


def evolve(ctx: Context, ham: Hamiltonian, psi: torch.Tensor, t0: float, t1: float, ws=None,
           carry=None, **kw):
    """Evolve psi in place from t0 to t1.  Returns (stats dict, recorded segments).
    carry (from new_carry()): continue a chain of fixed-step pc4 calls; psi is
    then left in the shifted frame, psi(t1) = complex(carry.phase_re,
    carry.phase_im) * psi, and the same workspace tensor must be passed again."""
    dt = _check_state(ctx, ham, psi)
    opts, keep, rec = evolve_opts(**kw)
    if carry is not None:
        opts.carry = C.pointer(carry)
    need = evolve_workspace_bytes(ham, dt, opts)
    if ws is None or ws.numel() < need:
        ws = workspace(ctx, need)
    st = L.EvolveStats()
    status = lib().aqc_evolve(ctx.handle, ham.handle, _ptr(psi), dt, float(t0), float(t1),
                              C.byref(opts), _ptr(ws), ws.numel(), C.byref(st))
    check(status)
    segs = None
    if rec is not None:
        segs = [tuple(r) for r in rec[:min(st.n_segments, rec.shape[0])]]
    return st.as_dict(), segs


def norm2(ctx, psi):
    out = C.c_double()
    check(lib().aqc_norm2_len(ctx.handle, _ptr(psi), dtype_code(psi), psi.numel(), C.byref(out)))
    return out.value


def overlap(ctx, phi, psi):
    re, im = C.c_double(), C.c_double()
    if phi.numel() != psi.numel() or phi.dtype != psi.dtype:
        raise ValueError("overlap of states of different shapes or types")
    check(lib().aqc_overlap_len(ctx.handle, _ptr(phi), _ptr(psi), dtype_code(psi), psi.numel(),
                                C.byref(re), C.byref(im)))
    return complex(re.value, im.value)


def _full_space_n(psi):
    """n of a 2^n-amplitude state (the C calls below take n, not a length)."""
    N = psi.numel()
    if N < 1 or N & (N - 1):
        raise ValueError(f"a full-space state has 2^n amplitudes, got {N}")
    if not psi.is_contiguous():
        raise ValueError("state must be contiguous")
    return N.bit_length() - 1


def fidelity_state(ctx, psi, phi):
    _full_space_n(psi)
    if phi.numel() != psi.numel() or phi.dtype != psi.dtype or phi.device != psi.device or not phi.is_contiguous():
        raise ValueError("target state must match the state's size, type and device")
    out = C.c_double()
    check(lib().aqc_fidelity(ctx.handle, _ptr(psi), dtype_code(psi), _full_space_n(psi),
                             L.TARGET_STATE, _ptr(phi), 0, C.byref(out)))
    return out.value


def fidelity_basis(ctx, psi, indices):
    idx = np.ascontiguousarray(np.asarray(indices, dtype=np.int64))
    out = C.c_double()
    check(lib().aqc_fidelity(ctx.handle, _ptr(psi), dtype_code(psi), _full_space_n(psi),
                             L.TARGET_BASIS_LIST, idx.ctypes.data_as(C.c_void_p), len(idx),
                             C.byref(out)))
    return out.value


def ground_mass(ctx, ham, t, psi, rel_tol=1e-9):
    _check_state(ctx, ham, psi)
    mass, emin = C.c_double(), C.c_double()
    check(lib().aqc_ground_mass(ctx.handle, ham.handle, float(t), _ptr(psi), dtype_code(psi),
                                float(rel_tol), C.byref(mass), C.byref(emin)))
    return mass.value, emin.value


def energy(ctx, ham, t, psi, ws=None):
    dt = _check_state(ctx, ham, psi)
    need = lib().aqc_apply_workspace_bytes(ham.handle, dt)
    if need and ws is None:
        ws = workspace(ctx, need)
    out = C.c_double()
    check(lib().aqc_energy(ctx.handle, ham.handle, float(t), _ptr(psi), dt,
                           _ptr(ws) if ws is not None else None, ws.numel() if ws is not None else 0,
                           C.byref(out)))
    return out.value


def energy_noalloc(ctx, ham, t, psi):
    """energy() without workspace or allocation (aqc_energy_noalloc): the
    library's fixed device scratch holds the intermediate vectors."""
    dt = _check_state(ctx, ham, psi)
    out = C.c_double()
    check(lib().aqc_energy_noalloc(ctx.handle, ham.handle, float(t), _ptr(psi), dt, C.byref(out)))
    return out.value


def lowest_eigs(ctx, ham, t, k=2, dtype=torch.complex128, max_basis=24, max_matvecs=4000, tol=1e-10,
                start=None, ws=None, ground=None):
    """The k smallest eigenvalues of H(t) (aqc_lowest_eigs).  Returns
    (eigenvalues, residual norms, products used); `ground` (a device state of
    the Hamiltonian's dimension and `dtype`) receives the lowest Ritz vector."""
    dt = L.C64 if dtype in (torch.complex64, L.C64) else L.C128
    need = lib().aqc_lowest_eigs_workspace_bytes(ham.handle, dt, int(max_basis))
    if need == 0:
        raise ValueError("bad max_basis for aqc_lowest_eigs")
    if ws is None or ws.numel() < need:
        ws = workspace(ctx, need)
    if start is not None:
        _check_state(ctx, ham, start)
        if start.dtype != dtype:
            raise ValueError("start must have the basis dtype")
    if ground is not None:
        _check_state(ctx, ham, ground)
        if ground.dtype != dtype:
            raise ValueError("ground must have the basis dtype")
    ev = (C.c_double * k)()
    rs = (C.c_double * k)()
    nmv = C.c_int()
    check(lib().aqc_lowest_eigs(ctx.handle, ham.handle, float(t), dt, int(k), int(max_basis),
                                int(max_matvecs), float(tol), _ptr(start) if start is not None else None,
                                _ptr(ws), ws.numel(), ev, rs, C.byref(nmv),
                                _ptr(ground) if ground is not None else None))
    return np.array(ev[:]), np.array(rs[:]), nmv.value


def hermitian_eigh(a):
    """Eigenvalues and eigenvectors of a small Hermitian matrix with the
    library's host solver (aqc_hermitian_eigh)."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    n = a.shape[0]
    w = np.zeros(n)
    z = np.zeros((n, n), dtype=np.complex128)
    dp = C.POINTER(C.c_double)
    check(lib().aqc_hermitian_eigh(n, a.view(np.float64).ctypes.data_as(dp), w.ctypes.data_as(dp),
                                   z.view(np.float64).ctypes.data_as(dp)))
    return w, z


def profile_enable(ctx, on=True):
    check(lib().aqc_profile_enable(ctx.handle, 1 if on else 0))


def profile_reset(ctx):
    check(lib().aqc_profile_reset(ctx.handle))


def profile_read(ctx):
    """{"high_pass": (ms, launches, bytes), "last_pass": (...)} since the last reset."""
    out = {}
    for name, kind in (("high_pass", L.PROF_HIGH_PASS), ("last_pass", L.PROF_LAST_PASS)):
        ms, n, b = C.c_double(), C.c_int64(), C.c_double()
        check(lib().aqc_profile_read(ctx.handle, kind, C.byref(ms), C.byref(n), C.byref(b)))
        out[name] = (ms.value, n.value, b.value)
    return out


class Batch:
    """Many fixed-step predictor-corrector solves advanced together (aqc_batch_*)."""

    def __init__(self, ctx: Context, dtype=torch.complex64, capacity=512, graph=True, resident_max_n=0):
        self.ctx = ctx
        self.dtype = dtype
        self.dt = L.C64 if dtype == torch.complex64 else L.C128
        h = C.c_void_p()
        check(lib().aqc_batch_create(ctx.handle, self.dt, int(capacity), C.byref(h)))
        self._h = h
        self.capacity = capacity
        self.set_graph(graph)
        self.set_resident(resident_max_n)
        self._keep = {}   # slot -> (psi, workspace, Hamiltonian) kept alive until retired

    def set_graph(self, on):
        check(lib().aqc_batch_set_graph(self._h, 1 if on else 0))

    def set_resident(self, max_n):
        """Solves admitted later with n <= max_n run as resident solves (one
        workgroup each, all steps in one launch); 0 turns it off."""
        check(lib().aqc_batch_set_resident(self._h, int(max_n)))

    def workspace_bytes(self, ham):
        return lib().aqc_batch_workspace_bytes(ham.handle, self.dt)

    def admit(self, ham, psi, t0, t1, n_steps, shift, ws=None):
        if psi.dtype != self.dtype:
            raise TypeError("state dtype differs from the batch dtype")
        _check_state(self.ctx, ham, psi)
        need = self.workspace_bytes(ham)
        if ws is None or ws.numel() < need:
            ws = workspace(self.ctx, need)
        slot = C.c_int()
        check(lib().aqc_batch_admit(self._h, ham.handle, _ptr(psi), _ptr(ws), ws.numel(), float(t0),
                                    float(t1), int(n_steps), float(shift), C.byref(slot)))
        self._keep[slot.value] = (psi, ws, ham)
        return slot.value

    def step(self, ticks=1):
        na = C.c_int()
        check(lib().aqc_batch_step(self._h, int(ticks), C.byref(na)))
        return na.value

    def poll(self):
        cap = self.capacity
        arr = (C.c_int * cap)()
        n = C.c_int()
        check(lib().aqc_batch_poll(self._h, arr, cap, C.byref(n)))
        return [arr[i] for i in range(n.value)]

    def retire(self, slot):
        st = L.EvolveStats()
        check(lib().aqc_batch_retire(self._h, int(slot), C.byref(st)))
        psi, ws, ham = self._keep.pop(slot)
        return psi, st.as_dict()

    def info(self):
        a, f, t = C.c_int(), C.c_int(), C.c_int64()
        check(lib().aqc_batch_info(self._h, C.byref(a), C.byref(f), C.byref(t)))
        return {"active": a.value, "finished": f.value, "ticks": t.value}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().aqc_batch_destroy(self._h)
            self._h = C.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
