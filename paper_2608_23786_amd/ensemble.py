"""Python face of the MI355X Monte Carlo KBC lattice Boltzmann library.

PyTorch supplies device memory (uint8 tensors the library borrows) and the
HIP stream; every step of the method runs in the library's kernels.
"""
import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

from . import _lib
from ._lib import MclbmError, SampleDesc, check, lib

PRECISIONS = {"f64": _lib.FP64, "f32s": _lib.FP32_SHIFTED}
RECORD_FIELDS = ("mass", "jx", "jy", "jz", "ke", "gamma_min", "gamma_max", "gamma_mean")


@dataclass
class Sample:
    n: int
    u0: float
    re: float
    amp: float = 0.0
    project: bool = False
    stride: int = 1

    def desc(self) -> SampleDesc:
        return SampleDesc(self.n, self.u0, self.re, self.amp, int(self.project), self.stride)


def omega(n: int, u0: float, re: float) -> float:
    """Shear relaxation frequency the library uses for a sample."""
    return lib().mclbm_omega(n, u0, re)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _require_cuda(t: torch.Tensor, dtype=None, numel=None, name="tensor"):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} needs at least {numel} elements")


class Ensemble:
    """An ensemble of RTGV samples evolved in one in-place population buffer."""

    def __init__(self, samples: Sequence[Sample], precision: str = "f32s", device="cuda:0",
                 stream: Optional[torch.cuda.Stream] = None, lattice: int = 27):
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {list(PRECISIONS)}")
        self.samples: List[Sample] = list(samples)
        self.m = len(self.samples)
        self.precision = precision
        self.q = int(lattice)   # 27 (D3Q27) or 19 (D3Q19); the library validates it
        self.device = torch.device(device)
        L = lib()
        self._desc = (SampleDesc * self.m)(*[s.desc() for s in self.samples])
        nbytes = L.mclbm_workspace_bytes(self.m, self._desc, PRECISIONS[precision], self.q)
        if nbytes == 0:
            # the library reports the reason of invalid descriptors on create
            nbytes = 256
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self._ctx = ctypes.c_void_p()
        check(L.mclbm_create(ctypes.byref(self._ctx), self.m, self._desc, PRECISIONS[precision], self.q,
                             ctypes.c_void_p(self._ws_ptr), nbytes, ctypes.c_void_p(self.stream.cuda_stream)))

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and ctx.value:
            try:
                lib().mclbm_destroy(ctx)
            except Exception:
                pass
            self._ctx = None

    # ------------------------------------------------------------ helpers
    def _dev_empty(self, shape, dtype=torch.float64):
        with torch.cuda.stream(self.stream):
            return torch.empty(shape, dtype=dtype, device=self.device)

    def synchronize(self):
        self.stream.synchronize()

    def _consume(self, *inputs):
        """The library's stream waits for work the caller queued on its current
        stream; caller tensors it reads or writes are marked as used on the
        library's stream, so that the caching allocator does not hand their
        memory out again before the library's work on them is done."""
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        for t in inputs:
            if t is not None:
                t.record_stream(self.stream)

    def _produce(self, *outputs):
        """The caller's current stream waits for the library's outputs, which
        are allocated on the library's stream and marked as used on the
        caller's stream too (freeing them there is then safe)."""
        cur = torch.cuda.current_stream(self.device)
        cur.wait_stream(self.stream)
        for t in outputs:
            if t is not None:
                t.record_stream(cur)

    # ------------------------------------------------------------ lifecycle
    def init(self, seed: int = 0, y: Optional[torch.Tensor] = None):
        if y is not None:
            yh = torch.as_tensor(y, dtype=torch.float64).contiguous().cpu()
            if yh.numel() != self.m * 24:
                raise ValueError("y must have m x 24 values")
            check(lib().mclbm_init(self._ctx, seed, ctypes.cast(yh.data_ptr(), _lib._dp)))
        else:
            check(lib().mclbm_init(self._ctx, seed, None))

    def y(self) -> torch.Tensor:
        out = torch.empty((self.m, 24), dtype=torch.float64)
        check(lib().mclbm_get_y(self._ctx, ctypes.cast(out.data_ptr(), _lib._dp)))
        return out

    def set_viscosity(self, eps: Sequence[float]):
        arr = (ctypes.c_double * self.m)(*eps)
        check(lib().mclbm_set_viscosity(self._ctx, arr))

    def step(self, ticks: int, record_every: int = 0) -> Optional[torch.Tensor]:
        if record_every > 0:
            nrec = (ticks + record_every - 1) // record_every
            rec = self._dev_empty((max(nrec, 1), self.m, 8))
            check(lib().mclbm_step(self._ctx, ticks, record_every, _ptr(rec), nrec))
            self._produce(rec)
            return rec[:nrec]
        check(lib().mclbm_step(self._ctx, ticks, 0, None, 0))
        return None

    @property
    def ticks(self) -> int:
        return int(lib().mclbm_ticks(self._ctx))

    def steps(self, sample: int) -> int:
        return int(lib().mclbm_steps(self._ctx, sample))

    # ------------------------------------------------------------ read-out
    def _check_sample(self, sample: int):
        if not 0 <= sample < self.m:
            # let the library report the error
            check(lib().mclbm_moments(self._ctx, sample, None, None))

    def moments(self, sample: int):
        self._check_sample(sample)
        n = self.samples[sample].n
        rho = self._dev_empty((n, n, n))
        u = self._dev_empty((3, n, n, n))
        check(lib().mclbm_moments(self._ctx, sample, _ptr(rho), _ptr(u)))
        self._produce(rho, u)
        return rho, u

    def reduce(self) -> torch.Tensor:
        red = self._dev_empty((self.m, 8))
        check(lib().mclbm_reduce(self._ctx, _ptr(red)))
        self._produce(red)
        return red

    def check(self) -> int:
        bad = ctypes.c_int32(-1)
        st = lib().mclbm_check(self._ctx, ctypes.byref(bad))
        if st not in (_lib.OK, _lib.ERR_UNSTABLE):
            check(st)
        return bad.value

    def get_state(self, sample: int) -> torch.Tensor:
        self._check_sample(sample)
        n = self.samples[sample].n
        f = self._dev_empty((self.q, n, n, n))
        check(lib().mclbm_get_state(self._ctx, sample, _ptr(f)))
        self._produce(f)
        return f

    def set_state(self, sample: int, f: torch.Tensor):
        self._check_sample(sample)
        n = self.samples[sample].n
        _require_cuda(f, torch.float64, self.q * n ** 3, "f")
        self._consume(f)
        check(lib().mclbm_set_state(self._ctx, sample, _ptr(f)))

    def observables(self, sample: int, work: Optional[torch.Tensor] = None, structure: bool = True,
                    spectrum: bool = True):
        """(S2[r = 1..n/2], E[kappa = 0..n/2]) of one sample's current state, float64 on the
        device; an observable not asked for is returned as None."""
        self._check_sample(sample)
        n = self.samples[sample].n
        wb = int(lib().mclbm_observables_work_bytes(self._ctx, sample))
        if work is None or work.numel() < wb:
            work = self._dev_empty((wb,), torch.uint8)
        s2 = self._dev_empty((n // 2,)) if structure else None
        ek = self._dev_empty((n // 2 + 1,)) if spectrum else None
        self._consume(work)
        check(lib().mclbm_observables(self._ctx, sample, _ptr(s2), _ptr(ek), _ptr(work), work.numel()))
        self._produce(s2, ek)
        return s2, ek

    def observables_range(self, first: int, count: int, work: Optional[torch.Tensor] = None, structure: bool = True,
                          spectrum: bool = True):
        """(S2[count, n/2], E[count, n/2+1]) of samples first..first+count-1 (one n) in one set of launches."""
        wb = int(lib().mclbm_observables_range_work_bytes(self._ctx, first, count))
        if wb == 0:
            raise MclbmError(_lib.ERR_ARG, "invalid sample range (out of bounds, mixed resolutions or n above 512)")
        n = self.samples[first].n
        if work is None or work.numel() < wb:
            work = self._dev_empty((wb,), torch.uint8)
        s2 = self._dev_empty((count, n // 2)) if structure else None
        ek = self._dev_empty((count, n // 2 + 1)) if spectrum else None
        self._consume(work)
        check(lib().mclbm_observables_range(self._ctx, first, count, _ptr(s2), _ptr(ek), _ptr(work), work.numel()))
        self._produce(s2, ek)
        return s2, ek

    def capture_velocity(self, enable: bool = True) -> Optional[torch.Tensor]:
        """While enabled, every record tick of step() also writes the float64
        velocity of the state it reads (the state its record describes) into a
        buffer the ensemble owns, which is returned: per sample three planes of
        n^3 one after another (velocity() gives one sample's view). Disabling
        clears the library's pointer before the buffer is released."""
        if not enable:
            check(lib().mclbm_capture_velocity(self._ctx, None, 0))
            self._vel = None
            return None
        nbytes = int(lib().mclbm_velocity_bytes(self._ctx))
        buf = self._dev_empty((nbytes // 8,))
        if buf.data_ptr() % 256:
            raise MclbmError(_lib.ERR_ARG, "the capture buffer is not 256-byte aligned")
        check(lib().mclbm_capture_velocity(self._ctx, _ptr(buf), nbytes))
        self._vel = buf
        return buf

    def velocity(self, sample: int) -> torch.Tensor:
        """[3, n, n, n] float64 view of one sample's captured velocity."""
        self._check_sample(sample)
        if getattr(self, "_vel", None) is None:
            raise MclbmError(_lib.ERR_STATE, "no velocity capture is set")
        off = sum(3 * s.n ** 3 for s in self.samples[:sample])
        n = self.samples[sample].n
        return self._vel[off:off + 3 * n ** 3].view(3, n, n, n)

    def observables_velocity_range(self, first: int, count: int, u: Optional[torch.Tensor] = None,
                                   work: Optional[torch.Tensor] = None, structure: bool = True,
                                   spectrum: bool = True):
        """observables_range() of the velocity fields in u (the capture layout;
        by default the capture buffer, i.e. the state the last record tick read)."""
        wb = int(lib().mclbm_observables_range_work_bytes(self._ctx, first, count))
        if wb == 0:
            raise MclbmError(_lib.ERR_ARG, "invalid sample range (out of bounds, mixed resolutions or n above 512)")
        if u is None:
            u = getattr(self, "_vel", None)
            if u is None:
                raise MclbmError(_lib.ERR_STATE, "no velocity capture is set")
        _require_cuda(u, torch.float64, sum(3 * s.n ** 3 for s in self.samples), "u")
        n = self.samples[first].n
        if work is None or work.numel() < wb:
            work = self._dev_empty((wb,), torch.uint8)
        s2 = self._dev_empty((count, n // 2)) if structure else None
        ek = self._dev_empty((count, n // 2 + 1)) if spectrum else None
        self._consume(work, u)
        check(lib().mclbm_observables_velocity_range(self._ctx, first, count, _ptr(u), _ptr(s2), _ptr(ek), _ptr(work),
                                                     work.numel()))
        self._produce(s2, ek)
        return s2, ek

    def point_values(self, q: int = 8, physical: bool = False) -> torch.Tensor:
        """Velocity at the q^3 nodes common to all resolutions: [m, 3, q^3] float64,
        in lattice units or, with physical, as u / u0."""
        out = self._dev_empty((self.m, 3, q ** 3))
        check(lib().mclbm_point_values(self._ctx, q, int(physical), _ptr(out)))
        self._produce(out)
        return out

    def get_cells(self, sample: int, cells) -> torch.Tensor:
        """Populations f[k][q] (float64, device) of the given cell indices of one sample."""
        idx = torch.as_tensor(cells, dtype=torch.int64).to(self.device).contiguous()
        out = self._dev_empty((idx.numel(), self.q))
        self._consume(idx)
        check(lib().mclbm_get_cells(self._ctx, sample, _ptr(idx), idx.numel(), _ptr(out)))
        self._produce(out)
        return out

    def poison(self, sample: int, cell: int, i: int):
        check(lib().mclbm_poison(self._ctx, sample, cell, i))

    # ------------------------------------------------------------ checkpoints
    def checkpoint_bytes(self) -> int:
        return int(lib().mclbm_checkpoint_bytes(self._ctx))

    def checkpoint(self, buf: Optional[torch.Tensor] = None) -> torch.Tensor:
        nb = self.checkpoint_bytes()
        if buf is None:
            buf = self._dev_empty((nb,), torch.uint8)
        self._consume(buf)
        check(lib().mclbm_checkpoint(self._ctx, _ptr(buf), buf.numel()))
        self._produce(buf)
        return buf

    def restore(self, buf: torch.Tensor):
        self._consume(buf)
        check(lib().mclbm_restore(self._ctx, _ptr(buf), buf.numel()))

    # ------------------------------------------------------------ launch shape
    def set_launch(self, block: int, xcd_remap: int = 0, buffer_addressing: int = 1, nontemporal: int = 1):
        check(lib().mclbm_set_launch(self._ctx, block, xcd_remap, buffer_addressing, nontemporal))

    def get_launch(self):
        v = [ctypes.c_int32() for _ in range(4)]
        check(lib().mclbm_get_launch(self._ctx, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def autotune(self, reps: int = 2):
        """Time every launch shape; returns (block, xcd_remap, buffer_addressing, nontemporal) chosen."""
        scratch = self._dev_empty((self.checkpoint_bytes(),), torch.uint8)
        v = [ctypes.c_int32() for _ in range(4)]
        check(lib().mclbm_autotune(self._ctx, reps, _ptr(scratch), scratch.numel(), *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def dissipation(self, records: torch.Tensor, first_tick: int, record_every: int, eta: bool = True):
        """Dissipation rate d[nrec, m] (physical units) and, when eta, the
        Kolmogorov length eta[nrec] from records [nrec, m, 8] of `step`."""
        _require_cuda(records, torch.float64, name="records")
        nrec = records.numel() // (self.m * 8)
        diss = self._dev_empty((nrec, self.m))
        et = self._dev_empty((nrec,)) if eta else None
        self._consume(records)
        check(lib().mclbm_dissipation(self._ctx, _ptr(records), nrec, first_tick, record_every, _ptr(diss),
                                      _ptr(et) if et is not None else None))
        self._produce(diss, et)
        return diss, et

    def dissipation_spectra(self, first: int, ek: torch.Tensor, first_tick: int, record_every: int,
                            eta: bool = True):
        """The paper's approximation of the dissipation rate, -d/dt of the
        summed shell spectrum: d[nrec, count] (physical units) and, when eta,
        the Kolmogorov length eta[nrec] from spectra ek[nrec, count, n/2+1] of
        samples first..first+count-1 (one n) saved every record_every ticks
        from first_tick."""
        _require_cuda(ek, torch.float64, name="ek")
        if ek.dim() != 3:
            raise ValueError("ek must be [nrec, count, n/2+1]")
        nrec, count = ek.shape[0], ek.shape[1]
        if not 0 <= first < self.m or ek.shape[2] != self.samples[first].n // 2 + 1:
            raise ValueError("ek rows must hold n/2+1 values of the range's resolution")
        diss = self._dev_empty((nrec, count))
        et = self._dev_empty((nrec,)) if eta else None
        self._consume(ek)
        check(lib().mclbm_dissipation_spectra(self._ctx, first, count, _ptr(ek), nrec, first_tick, record_every,
                                              _ptr(diss), _ptr(et) if et is not None else None))
        self._produce(diss, et)
        return diss, et

    def compensate(self, first: int, diss: torch.Tensor, s2: Optional[torch.Tensor] = None,
                   ek: Optional[torch.Tensor] = None):
        """Sample-wise compensated structure functions [count, n/2] and spectra
        [count, n/2+1] of samples first.. (one n; count = len(diss)) from their
        dissipation rates diss[count] at the same time; velocities in units of
        u0. Returns (s2c, ekc), None where the input is None."""
        _require_cuda(diss, torch.float64, name="diss")
        count = diss.numel()
        n = self.samples[first].n if 0 <= first < self.m else 0
        for t, w, name in ((s2, n // 2, "s2"), (ek, n // 2 + 1, "ek")):
            if t is not None:
                _require_cuda(t, torch.float64, count * w, name)
        s2c = self._dev_empty((count, n // 2)) if s2 is not None else None
        ekc = self._dev_empty((count, n // 2 + 1)) if ek is not None else None
        self._consume(diss, s2, ek)
        check(lib().mclbm_compensate(self._ctx, first, count, _ptr(diss), _ptr(s2), _ptr(ek), _ptr(s2c), _ptr(ekc)))
        self._produce(s2c, ekc)
        return s2c, ekc

    def set_stabiliser(self, mode: str):
        """'closed_form' (eq. (entropyControl), default) or 'exact' (minimiser of
        the discrete H-function, eq. (kbc_entropy))."""
        modes = {"closed_form": _lib.GAMMA_CLOSED_FORM, "exact": _lib.GAMMA_EXACT}
        if mode not in modes:
            raise ValueError(f"stabiliser must be one of {list(modes)}")
        check(lib().mclbm_set_stabiliser(self._ctx, modes[mode]))

    def use_graphs(self, enable: bool):
        check(lib().mclbm_use_graphs(self._ctx, int(enable)))

    def time_launches(self, enable: bool):
        check(lib().mclbm_time_launches(self._ctx, int(enable)))

    def launch_time(self):
        avg = ctypes.c_double()
        cnt = ctypes.c_int64()
        check(lib().mclbm_launch_time(self._ctx, ctypes.byref(avg), ctypes.byref(cnt)))
        return avg.value, cnt.value

    # ------------------------------------------------------------ adjoint
    def forward_ckpt(self, ticks: int, ckpt_every: int) -> torch.Tensor:
        nb = int(lib().mclbm_ckpt_bytes(self._ctx, ticks, ckpt_every))
        if nb == 0:
            raise MclbmError(_lib.ERR_ARG, "invalid ticks / ckpt_every")
        ck = self._dev_empty((nb,), torch.uint8)
        check(lib().mclbm_forward_ckpt(self._ctx, ticks, ckpt_every, _ptr(ck), nb))
        self._produce(ck)
        return ck

    def step_vjp(self, lam: torch.Tensor) -> torch.Tensor:
        """One step's vector-Jacobian product at the current state of every
        sample: (d f_{n+1} / d f_n)^T lam. lam: float64 on the device, the
        samples one after another, each [q, n^3] in the order of get_state."""
        total = sum(self.q * s.n ** 3 for s in self.samples)
        _require_cuda(lam, torch.float64, numel=total, name="lam")
        wb = int(lib().mclbm_step_vjp_work_bytes(self._ctx))
        work = self._dev_empty((wb,), torch.uint8)
        out = self._dev_empty((total,))
        self._consume(lam)
        check(lib().mclbm_step_vjp(self._ctx, _ptr(lam), _ptr(out), _ptr(work), wb))
        self._produce(out)
        return out

    def backward(self, ticks: int, ckpt_every: int, ckpt: torch.Tensor):
        wb = int(lib().mclbm_backward_work_bytes(self._ctx, ckpt_every))
        work = self._dev_empty((wb,), torch.uint8)
        dj = self._dev_empty((self.m, 24))
        ke = self._dev_empty((self.m,))
        self._consume(ckpt)
        check(lib().mclbm_backward(self._ctx, ticks, ckpt_every, _ptr(ckpt), ckpt.numel(), _ptr(work), wb,
                                   _ptr(dj), _ptr(ke)))
        self._produce(dj, ke)
        return dj, ke


def _on_stream(stream: Optional[torch.cuda.Stream], *tensors) -> torch.cuda.Stream:
    """The stream a module-level call runs on (default: the current one). A
    different stream first waits for the current one, and the caller's
    tensors are marked as used on it."""
    cur = torch.cuda.current_stream()
    if stream is None or stream == cur:
        return cur
    stream.wait_stream(cur)
    for t in tensors:
        t.record_stream(stream)
    return stream


def w1_1pt(a: torch.Tensor, b: torch.Tensor, q: int = 8, stream: Optional[torch.cuda.Stream] = None):
    """Per-component terms of W_{1,1} between two ensembles' point values
    ([m, 3, q^3] float64 each); their sum is W_{1,1}."""
    _require_cuda(a, torch.float64, name="a")
    _require_cuda(b, torch.float64, name="b")
    if a.shape != b.shape or a.dim() != 3 or a.shape[1] != 3 or a.shape[2] != q ** 3:
        raise ValueError("a and b must both have shape [m, 3, q^3]")
    s = _on_stream(stream, a, b)
    wb = int(lib().mclbm_w1_work_bytes(q))
    with torch.cuda.stream(s):
        work = torch.empty(wb, dtype=torch.uint8, device=a.device)
        out = torch.empty(3, dtype=torch.float64, device=a.device)
    check(lib().mclbm_w1_1pt(_ptr(a), _ptr(b), a.shape[0], q, _ptr(out), _ptr(work), wb,
                             ctypes.c_void_p(s.cuda_stream)))
    return out


def ensemble_moments(x: torch.Tensor, std: bool = True, stream: Optional[torch.cuda.Stream] = None):
    """Empirical mean and standard deviation (1/(m-1)) over the rows of
    x [m, k] (float64 on the device, unit stride along k; rows may be strided,
    e.g. records[t, :, 4:5]). Returns (mean[k], std[k] or None)."""
    if not x.is_cuda or x.dtype != torch.float64 or x.dim() != 2 or (x.shape[1] > 1 and x.stride(1) != 1):
        raise ValueError("x must be a 2-D float64 device tensor with unit stride along its second axis")
    m, k = x.shape
    ld = x.stride(0) if m > 1 else k
    s = _on_stream(stream, x)
    with torch.cuda.stream(s):
        mean = torch.empty(k, dtype=torch.float64, device=x.device)
        sd = torch.empty(k, dtype=torch.float64, device=x.device) if std else None
    check(lib().mclbm_ensemble_moments(_ptr(x), m, k, ld, _ptr(mean), _ptr(sd), ctypes.c_void_p(s.cuda_stream)))
    return mean, sd


def sample_error(a: torch.Tensor, b: torch.Tensor, q: int = 8, stream: Optional[torch.cuda.Stream] = None):
    """Ensemble-mean relative L1 error of the samples of a against those of
    the reference b (point values [m, 3, q^3] float64 each, sample m of both
    from the same Y_m): components x, y, z and the velocity vector."""
    _require_cuda(a, torch.float64, name="a")
    _require_cuda(b, torch.float64, name="b")
    if a.shape != b.shape or a.dim() != 3 or a.shape[1] != 3 or a.shape[2] != q ** 3:
        raise ValueError("a and b must both have shape [m, 3, q^3]")
    s = _on_stream(stream, a, b)
    wb = int(lib().mclbm_sample_error_work_bytes(a.shape[0]))
    with torch.cuda.stream(s):
        work = torch.empty(wb, dtype=torch.uint8, device=a.device)
        out = torch.empty(4, dtype=torch.float64, device=a.device)
    check(lib().mclbm_sample_error(_ptr(a), _ptr(b), a.shape[0], q, _ptr(out), _ptr(work), wb,
                                   ctypes.c_void_p(s.cuda_stream)))
    return out


def eoc_slope(ns, ds) -> float:
    """Least-squares slope of log d over log n (host only)."""
    if len(ns) != len(ds):
        raise ValueError("ns and ds must have the same length")
    n = (ctypes.c_double * len(ns))(*[float(v) for v in ns])
    d = (ctypes.c_double * len(ds))(*[float(v) for v in ds])
    out = ctypes.c_double()
    check(lib().mclbm_eoc_slope(ctypes.cast(n, ctypes.c_void_p), ctypes.cast(d, ctypes.c_void_p), len(ns),
                                ctypes.byref(out)))
    return out.value


def stream_copy(dst: torch.Tensor, src: torch.Tensor, stream: Optional[torch.cuda.Stream] = None):
    nbytes = min(dst.numel() * dst.element_size(), src.numel() * src.element_size()) // 16 * 16
    s = _on_stream(stream, dst, src)
    check(lib().mclbm_stream_copy(_ptr(dst), _ptr(src), nbytes, ctypes.c_void_p(s.cuda_stream)))


class EnsembleKE(torch.autograd.Function):
    """J(Y) = (1/M) sum_m KE_m(T) for an ensemble started from Y.

    forward(Y, ensemble, ticks, ckpt_every) -> J (0-d float64 tensor);
    backward gives dJ/dY from the library's discrete adjoint."""

    @staticmethod
    def forward(ctx, y, ensemble: Ensemble, ticks: int, ckpt_every: int):
        ensemble.init(0, y.detach().cpu())
        ck = ensemble.forward_ckpt(ticks, ckpt_every)
        ctx.ensemble = ensemble
        ctx.y_device = y.device
        ctx.ticks = ticks
        ctx.ckpt_every = ckpt_every
        ctx.ckpt = ck
        red = ensemble.reduce()
        mean, _ = ensemble_moments(red[:, 4:5], std=False)
        ensemble.synchronize()
        return mean[0].to(y.device)

    @staticmethod
    def backward(ctx, gJ):
        dj, _ = ctx.ensemble.backward(ctx.ticks, ctx.ckpt_every, ctx.ckpt)
        ctx.ensemble.synchronize()
        ctx.ckpt = None
        return (gJ.to(dj.device) * dj).to(ctx.y_device), None, None, None
