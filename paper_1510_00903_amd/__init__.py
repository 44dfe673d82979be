"""MI355X effective-block baryon-baryon correlator: Python binding of libbbcorr.

The binding only marshals arguments for the C ABI declared in
``include/bbcorr.h``; every step of the computation runs in the HIP kernels of
``libbbcorr.so``.  PyTorch provides device memory and the current HIP stream.
There is no fallback: if the library is missing, every call raises.

Paper: H. Nemura, "Instructive discussion of an effective block algorithm for
baryon-baryon correlators", arXiv:1510.00903.
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["BBCError", "F64", "F32", "UPPER", "LOWER", "FULL", "STAGES", "CUBIC_A1", "CUBIC_A1_COMPLEMENT",
           "baryon_names", "channel_id",
           "Context", "library_path", "load",
           "num_channels", "num_channels_all", "channel_name", "channel_content", "source_terms",
           "diagram_table", "plan_stats", "footprint", "EXPORTED_SYMBOLS"]

F64, F32 = 0, 1
UPPER, LOWER, FULL = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libbbcorr.so")
_lib = None

EXPORTED_SYMBOLS = [
    "bbc_num_channels", "bbc_num_channels_all", "bbc_channel_name", "bbc_channel_content",
    "bbc_source_terms", "bbc_diagram_table", "bbc_plan_stats", "bbc_pair_stats", "bbc_create", "bbc_destroy",
    "bbc_last_error", "bbc_footprint", "bbc_correlate", "bbc_correlate_noalloc", "bbc_profile_enable",
    "bbc_profile_read",
    "bbc_server_start", "bbc_server_stop", "bbc_prop_upload", "bbc_prop_release", "bbc_submit", "bbc_poll",
    "bbc_wait", "bbc_cancel", "bbc_job_times", "bbc_job_forget",
    "bbc_spin_project", "bbc_cubic_project", "bbc_central_potential",
    "bbc_num_baryons", "bbc_baryon_name", "bbc_channel_id", "bbc_graph_mode", "bbc_correlate_cpt",
    "bbc_tuning_get", "bbc_tuning_set", "bbc_autotune", "bbc_tuning_save", "bbc_tuning_load",
]
CUBIC_A1, CUBIC_A1_COMPLEMENT = 0, 1
JOB_STATES = ["queued", "running", "done", "cancelled", "failed"]
ETIMEOUT, ECANCELLED, ESTATE, ENOMEM = -5, -6, -7, -2
STAGES = ["blocks", "fft_forward", "transpose", "contract", "fft_inverse", "finalize", "combine"]


class BBCError(RuntimeError):
    """A negative bbc_status from the library, with its message."""

    def __init__(self, msg, status=None):
        super().__init__(msg)
        self.status = status


def library_path() -> str:
    return _LIB_PATH


def load():
    """Load libbbcorr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise BBCError("libbbcorr.so is not built; run `python -m paper_1510_00903_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    I, P, I64, U64 = ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64
    lib.bbc_num_channels.restype = I
    lib.bbc_num_baryons.restype = I
    lib.bbc_baryon_name.argtypes = [I]
    lib.bbc_baryon_name.restype = ctypes.c_char_p
    lib.bbc_channel_id.argtypes = [I, I, I, I]
    lib.bbc_channel_id.restype = I
    lib.bbc_num_channels_all.restype = I
    lib.bbc_channel_name.argtypes = [I]
    lib.bbc_channel_name.restype = ctypes.c_char_p
    lib.bbc_channel_content.argtypes = [I, P, P]
    lib.bbc_source_terms.argtypes = [I, P, P]
    lib.bbc_diagram_table.argtypes = [I, I, I, I, P, P, P]
    lib.bbc_plan_stats.argtypes = [I, P, P, P, P, P]
    lib.bbc_pair_stats.argtypes = [I, P, P, P, P, P]
    lib.bbc_create.argtypes = [I, U64, P]
    lib.bbc_destroy.argtypes = [P]
    lib.bbc_destroy.restype = None
    lib.bbc_last_error.restype = ctypes.c_char_p
    lib.bbc_footprint.argtypes = [P, I, I, P, P]
    lib.bbc_correlate.argtypes = [P, P, I, P, P, I, P, I, I, P, I, P, P, P, P]
    lib.bbc_correlate_noalloc.argtypes = [P, P, I, P, P, I, P, I, I, P, I, P, P, P, P]
    lib.bbc_tuning_get.argtypes = [P, P, I, I, P, I, P, P]
    lib.bbc_tuning_set.argtypes = [P, P, I, I, P, I, P]
    lib.bbc_autotune.argtypes = [P, P, I, P, P, I, P, I, I, P, P, P]
    lib.bbc_tuning_save.argtypes = [P, ctypes.c_char_p]
    lib.bbc_tuning_load.argtypes = [P, ctypes.c_char_p]
    lib.bbc_correlate_cpt.argtypes = [P, P, I, I, P, P, I, I, P, I, P, I, P, P, P, P]
    lib.bbc_profile_enable.argtypes = [P, I]
    lib.bbc_profile_read.argtypes = [P, I, P, P]
    lib.bbc_graph_mode.argtypes = [P, I]
    lib.bbc_graph_mode.restype = I
    lib.bbc_server_start.argtypes = [P, I]
    lib.bbc_server_stop.argtypes = [P]
    lib.bbc_prop_upload.argtypes = [P, P, I, P, P, I, P]
    lib.bbc_prop_release.argtypes = [P, U64]
    lib.bbc_submit.argtypes = [P, U64, I, P, P, I, I, P, I, P, P, P, P]
    lib.bbc_poll.argtypes = [P, U64, P]
    lib.bbc_wait.argtypes = [P, U64, I]
    lib.bbc_cancel.argtypes = [P, U64]
    lib.bbc_job_times.argtypes = [P, U64, P, P, P]
    lib.bbc_job_forget.argtypes = [P, U64]
    lib.bbc_spin_project.argtypes = [P, P, I, I, P, I, P, P, P]
    lib.bbc_cubic_project.argtypes = [P, P, I, I, I, P, I, P, P]
    lib.bbc_central_potential.argtypes = [P, P, I, I, P, ctypes.c_double, P, P]
    for f in ("bbc_spin_project", "bbc_cubic_project", "bbc_central_potential", "bbc_channel_content", "bbc_source_terms", "bbc_diagram_table", "bbc_plan_stats", "bbc_pair_stats", "bbc_create",
              "bbc_footprint", "bbc_correlate", "bbc_correlate_noalloc", "bbc_profile_enable", "bbc_profile_read",
              "bbc_server_start", "bbc_server_stop", "bbc_prop_upload", "bbc_prop_release", "bbc_submit",
              "bbc_poll", "bbc_wait", "bbc_cancel", "bbc_job_times", "bbc_job_forget", "bbc_tuning_get",
              "bbc_tuning_set", "bbc_autotune", "bbc_tuning_save", "bbc_tuning_load"):
        getattr(lib, f).restype = I
    _lib = lib
    return lib


def _check(status):
    if status != 0:
        raise BBCError("bbcorr error %d: %s" % (status, load().bbc_last_error().decode()), status)


def _i32(values):
    vals = [int(v) for v in values]
    return (ctypes.c_int32 * max(1, len(vals)))(*vals), len(vals)


def _check_tensor(t, shape, dtype, name, device=None, host_ok=False):
    """Raise unless t is a contiguous tensor of this shape and dtype on `device`
    (or in host memory where host_ok): the library writes through raw pointers,
    so a wrong buffer would be written past its end on the GPU."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise BBCError("%s must be a torch tensor" % name)
    if tuple(t.shape) != tuple(int(v) for v in shape):
        raise BBCError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    if t.dtype != dtype:
        raise BBCError("%s has dtype %s, expected %s" % (name, t.dtype, dtype))
    if not t.is_contiguous():
        raise BBCError("%s must be contiguous" % name)
    if t.is_cuda:
        if device is not None and t.device != device:
            raise BBCError("%s is on %s, expected %s" % (name, t.device, device))
    elif not host_ok:
        raise BBCError("%s must be a device tensor" % name)


def _prop_dtype(S, name):
    import torch
    if S.dtype not in (torch.complex128, torch.complex64):
        raise BBCError("%s must be complex128 or complex64" % name)
    if S.dim() != 6 or tuple(S.shape[-2:]) != (12, 12):
        raise BBCError("%s must be [n_t, Lz, Ly, Lx, 12, 12]" % name)
    return F64 if S.dtype == torch.complex128 else F32


def num_channels() -> int:
    return load().bbc_num_channels()


def num_channels_all() -> int:
    return load().bbc_num_channels_all()


def channel_name(c: int) -> str:
    s = load().bbc_channel_name(c)
    if s is None:
        raise BBCError("invalid channel %d" % c)
    return s.decode()


def channel_content(c: int):
    nl, ns = ctypes.c_int(), ctypes.c_int()
    _check(load().bbc_channel_content(c, ctypes.byref(nl), ctypes.byref(ns)))
    return nl.value, ns.value


def source_terms(c: int):
    a, b = ctypes.c_int(), ctypes.c_int()
    _check(load().bbc_source_terms(c, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def diagram_table(c: int, term3: int, term4: int):
    """[(K, sign)] of every diagram of channel c for the given source terms."""
    K = (ctypes.c_int32 * 64)()
    sg = (ctypes.c_int32 * 64)()
    n = ctypes.c_int()
    _check(load().bbc_diagram_table(c, term3, term4, 64, ctypes.byref(n), K, sg))
    return [(K[i], sg[i]) for i in range(n.value)]


def baryon_names():
    """The fields that name channels, in index order: the octet p n S+ S- X0 X- L S0, then
    p2 n2 ({C, gamma_5} nucleon) and the decuplet D++ D- O- D+ D0 S*+ S*0 S*- X*0 X*-,
    each as name(l) for l = 1, 2, 3."""
    lib = load()
    return [lib.bbc_baryon_name(b).decode() for b in range(lib.bbc_num_baryons())]


def channel_id(b1, b2, b3, b4):
    """Channel index of the quadruple B1 B2 > B3 B4 (names or indices); other charge
    states than the 52 listed channels get extended ids."""
    names = baryon_names()
    idx = [names.index(b) if isinstance(b, str) else int(b) for b in (b1, b2, b3, b4)]
    c = load().bbc_channel_id(*idx)
    if c < 0:
        _check(c)
    return c


def plan_stats(channels):
    arr, n = _i32(channels)
    vals = [ctypes.c_int64() for _ in range(4)]
    _check(load().bbc_plan_stats(n, arr, *[ctypes.byref(v) for v in vals]))
    keys = ("intermediates", "components", "diagrams", "iterations")
    return dict(zip(keys, (v.value for v in vals)))


def pair_stats(channels):
    """Pair form of the contraction: distinct pair products, tasks, sum of K over
    pairs, (channel, pair) weights."""
    arr, n = _i32(channels)
    vals = [ctypes.c_int64() for _ in range(4)]
    _check(load().bbc_pair_stats(n, arr, *[ctypes.byref(v) for v in vals]))
    keys = ("pairs", "tasks", "pair_items", "weights")
    return dict(zip(keys, (v.value for v in vals)))


def footprint(lattice, channels, precision=F64) -> int:
    lat, _ = _i32(lattice)
    arr, n = _i32(channels)
    b = ctypes.c_uint64()
    _check(load().bbc_footprint(lat, precision, n, arr, ctypes.byref(b)))
    return b.value


class _Tuning(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_int32), ("blocks", ctypes.c_int32), ("planes", ctypes.c_int32),
                ("slices", ctypes.c_int32), ("combine", ctypes.c_int32)]


class Context:
    """A device context: plan cache and workspace on one GPU."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self._lib = load()
        self._ptr = ctypes.c_void_p()
        _check(self._lib.bbc_create(device, hbm_budget_bytes, ctypes.byref(self._ptr)))
        self.device = device
        self._props = {}           # handle -> (n_t, Lz, Ly, Lx, dtype) of a resident propagator set

    def _torch_device(self):
        import torch
        return torch.device("cuda", self.device)

    def close(self):
        if self._ptr:
            self._lib.bbc_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, enable: bool = True):
        """Record HIP events around every kernel stage of later correlate calls."""
        _check(self._lib.bbc_profile_enable(self._ptr, 1 if enable else 0))

    def graph_mode(self, enable: bool = True):
        """Capture device-resident correlate calls into cached HIP graphs and replay them."""
        _check(self._lib.bbc_graph_mode(self._ptr, 1 if enable else 0))

    def profile_read(self):
        """{stage: (milliseconds, launches)} accumulated since the last read."""
        n = len(STAGES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        _check(self._lib.bbc_profile_read(self._ptr, n, ms, cnt))
        return {STAGES[i]: (ms[i], cnt[i]) for i in range(n)}

    # ---------------------------------------------------------------- serving
    def server_start(self, n_slots: int = 2):
        """Start the continuous-batching scheduler with n_slots concurrent job slots."""
        _check(self._lib.bbc_server_start(self._ptr, n_slots))

    def server_stop(self):
        _check(self._lib.bbc_server_stop(self._ptr))

    def prop_upload(self, S_light, S_strange) -> int:
        """Copy a propagator set ([n_t, Lz, Ly, Lx, 12, 12] complex, host or device tensors)
        into memory owned by the context; returns its handle."""
        if S_light.shape != S_strange.shape or S_light.dtype != S_strange.dtype:
            raise BBCError("S_light and S_strange must have the same shape and dtype")
        prec = _prop_dtype(S_light, "S_light")
        for S, nm in ((S_light, "S_light"), (S_strange, "S_strange")):
            if S.is_cuda and S.device != self._torch_device():
                raise BBCError("%s is on %s, the context on cuda:%d" % (nm, S.device, self.device))
        S_light, S_strange = S_light.contiguous(), S_strange.contiguous()
        n_t, Lz, Ly, Lx = S_light.shape[:4]
        lat, _ = _i32([Lx, Ly, Lz])
        h = ctypes.c_uint64()
        _check(self._lib.bbc_prop_upload(self._ptr, lat, prec, ctypes.c_void_p(S_light.data_ptr()),
                                         ctypes.c_void_p(S_strange.data_ptr()), n_t, ctypes.byref(h)))
        self._props[h.value] = (n_t, Lz, Ly, Lx, S_light.dtype)
        return h.value

    def prop_release(self, handle: int):
        _check(self._lib.bbc_prop_release(self._ptr, handle))
        self._props.pop(handle, None)

    def submit(self, prop: int, slices, t_list, channels, out, scale=None, t0=0, spin=UPPER, energy=None) -> int:
        """Queue a job over slices of a resident propagator set; out (and scale in FP32)
        are caller-owned device tensors shaped as for correlate()."""
        import torch
        s_arr, n_t = _i32(slices)
        t_arr, n2 = _i32(t_list)
        ch_arr, n_ch = _i32(channels)
        if n2 != n_t:
            raise BBCError("t_list must have one entry per slice")
        if prop not in self._props:
            raise BBCError("unknown propagator handle %d" % prop)
        _, Lz, Ly, Lx, dt = self._props[prop]
        dev = self._torch_device()
        _check_tensor(out, (n_t, n_ch, Lz, Ly, Lx, 16), dt, "out", dev)
        if dt == torch.complex64:
            if scale is None:
                raise BBCError("scale is required in the FP32 form")
            _check_tensor(scale, (n_t, n_ch), torch.float64, "scale", dev)
        else:
            scale = None
        e_arr = None
        if energy is not None:
            e_arr = (ctypes.c_double * n_ch)(*[float(e) for e in energy])
        j = ctypes.c_uint64()
        _check(self._lib.bbc_submit(self._ptr, prop, n_t, s_arr, t_arr, int(t0), n_ch, ch_arr, int(spin), e_arr,
                                    ctypes.c_void_p(out.data_ptr()),
                                    ctypes.c_void_p(scale.data_ptr()) if scale is not None else None,
                                    ctypes.byref(j)))
        return j.value

    def poll(self, job: int) -> str:
        st = ctypes.c_int()
        _check(self._lib.bbc_poll(self._ptr, job, ctypes.byref(st)))
        return JOB_STATES[st.value]

    def wait(self, job: int, timeout_ms: int = -1):
        _check(self._lib.bbc_wait(self._ptr, job, timeout_ms))

    def cancel(self, job: int):
        _check(self._lib.bbc_cancel(self._ptr, job))

    def job_times(self, job: int):
        """(queue_ms, run_ms, total_ms) of a finished job."""
        v = [ctypes.c_double() for _ in range(3)]
        _check(self._lib.bbc_job_times(self._ptr, job, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def job_forget(self, job: int):
        _check(self._lib.bbc_job_forget(self._ptr, job))

    def correlate(self, S_light, S_strange, t_list, channels, t0=0, spin=UPPER, energy=None, out=None,
                  scale=None, stream=None):
        """C_ch(r, t) for the slices in S_light/S_strange.

        S_*:   [n_t, Lz, Ly, Lx, 12, 12], complex128 (FP64 form) or complex64 (FP32 form), on the
               context's GPU or in host memory (pinned recommended: slices are then streamed
               through device staging buffers, overlapping the transfers with the kernels).
        spin:  UPPER, LOWER, or FULL (all 256 components, alpha + 4 (beta + 4 (alpha' + 4 beta')),
               output on the device only).
        out:   device or host tensor (default: device if the inputs are or spin is FULL, else
               pinned host memory).
        Returns ``out`` [n_t, n_ch, Lz, Ly, Lx, 16] (256 for FULL, same dtype); in the FP32 form
        also ``scale`` [n_t, n_ch] float64, the FP64 factor of each (t, channel) field.
        Stream-ordered on ``stream`` (default: torch's current stream).
        """
        import torch

        if S_light.shape != S_strange.shape or S_light.dtype != S_strange.dtype:
            raise BBCError("S_light and S_strange must have the same shape and dtype")
        prec = _prop_dtype(S_light, "propagators")
        if S_light.is_cuda != S_strange.is_cuda:
            raise BBCError("S_light and S_strange must both be on the device or both on the host")
        if S_light.is_cuda and S_light.device != self._torch_device():
            raise BBCError("propagators are on %s, the context on cuda:%d" % (S_light.device, self.device))
        S_light = S_light.contiguous()
        S_strange = S_strange.contiguous()
        n_t, Lz, Ly, Lx = S_light.shape[:4]
        t_arr, nt2 = _i32(t_list)
        if nt2 != n_t:
            raise BBCError("t_list must have one entry per slice")
        ch_arr, n_ch = _i32(channels)
        lat, _ = _i32([Lx, Ly, Lz])
        dev = self._torch_device()
        full = int(spin) == FULL
        oshape = (n_t, n_ch, Lz, Ly, Lx, 256 if full else 16)
        if out is None:
            if S_light.is_cuda or full:
                out = torch.empty(oshape, dtype=S_light.dtype, device=dev)
            else:
                out = torch.empty(oshape, dtype=S_light.dtype, pin_memory=True)
        _check_tensor(out, oshape, S_light.dtype, "out", dev, host_ok=not full)
        if prec == F32:
            if scale is None:
                scale = torch.empty((n_t, n_ch), dtype=torch.float64, device=dev)
            _check_tensor(scale, (n_t, n_ch), torch.float64, "scale", dev)
        e_arr = None
        if energy is not None:
            e_vals = [float(e) for e in energy]
            if len(e_vals) != n_ch:
                raise BBCError("energy must have one entry per channel")
            e_arr = (ctypes.c_double * n_ch)(*e_vals)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        _check(self._lib.bbc_correlate(
            self._ptr, lat, prec, ctypes.c_void_p(S_light.data_ptr()), ctypes.c_void_p(S_strange.data_ptr()),
            n_t, t_arr, int(t0), n_ch, ch_arr, int(spin), e_arr, ctypes.c_void_p(out.data_ptr()),
            ctypes.c_void_p(scale.data_ptr()) if (prec == F32) else None,
            ctypes.c_void_p(stream.cuda_stream)))
        return (out, scale) if prec == F32 else out

    # -- kernel variants of a request shape (bbc_tuning_*, bbc_autotune) ----------
    def tuning(self, lattice, channels, precision=F64, spin=UPPER):
        """Kernel variants of a request shape: (dict pairs/blocks/planes, tuned?)."""
        lat, _ = _i32(lattice)
        arr, n = _i32(channels)
        t = _Tuning()
        tuned = ctypes.c_int()
        _check(self._lib.bbc_tuning_get(self._ptr, lat, int(precision), n, arr, int(spin), ctypes.byref(t),
                                        ctypes.byref(tuned)))
        return {"pairs": t.pairs, "blocks": t.blocks, "planes": t.planes, "slices": t.slices,
                "combine": t.combine}, bool(tuned.value)

    def set_tuning(self, lattice, channels, tuning, precision=F64, spin=UPPER):
        """Set the variants of a request shape (dict pairs/blocks/planes/slices/combine; None: built-in)."""
        lat, _ = _i32(lattice)
        arr, n = _i32(channels)
        t = None
        if tuning is not None:
            t = ctypes.byref(_Tuning(int(tuning["pairs"]), int(tuning["blocks"]), int(tuning["planes"]),
                                     int(tuning.get("slices", 0)), int(tuning.get("combine", 0))))
        _check(self._lib.bbc_tuning_set(self._ptr, lat, int(precision), n, arr, int(spin), t))

    def autotune(self, S_light, S_strange, channels, spin=UPPER, reps=3, stream=None):
        """Time the kernel variants on one device-resident slice ([Lz, Ly, Lx, 12, 12]) and keep
        the fastest; returns (dict pairs/blocks/planes, ms per slice)."""
        import torch

        if S_light.shape != S_strange.shape or S_light.dtype != S_strange.dtype:
            raise BBCError("S_light and S_strange must have the same shape and dtype")
        prec = _prop_dtype(S_light.unsqueeze(0), "propagators")
        dev = self._torch_device()
        for name, s in (("S_light", S_light), ("S_strange", S_strange)):
            if not s.is_cuda or s.device != dev or not s.is_contiguous():
                raise BBCError("%s must be a contiguous tensor on cuda:%d" % (name, self.device))
        Lz, Ly, Lx = S_light.shape[:3]
        lat, _ = _i32([Lx, Ly, Lz])
        arr, n = _i32(channels)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        t = _Tuning()
        ms = ctypes.c_double()
        _check(self._lib.bbc_autotune(self._ptr, lat, prec, ctypes.c_void_p(S_light.data_ptr()),
                                      ctypes.c_void_p(S_strange.data_ptr()), n, arr, int(spin), int(reps),
                                      ctypes.c_void_p(stream.cuda_stream), ctypes.byref(t), ctypes.byref(ms)))
        return {"pairs": t.pairs, "blocks": t.blocks, "planes": t.planes, "slices": t.slices,
                "combine": t.combine}, ms.value

    def save_tuning(self, path):
        _check(self._lib.bbc_tuning_save(self._ptr, os.fsencode(path)))

    def load_tuning(self, path):
        _check(self._lib.bbc_tuning_load(self._ptr, os.fsencode(path)))

    def correlate_noalloc(self, S_light, S_strange, t_list, channels, out, scale=None, t0=0, spin=UPPER,
                          energy=None, stream=None):
        """correlate() through bbc_correlate_noalloc: no device allocation by the library
        (its tables and workspace live in a fixed 192 MiB scratch array per GPU).
        Device tensors only; ``out`` (and ``scale`` in the FP32 form) are required.
        Returns ``out`` (FP64) or ``(out, scale)`` (FP32)."""
        import torch

        if S_light.shape != S_strange.shape or S_light.dtype != S_strange.dtype:
            raise BBCError("S_light and S_strange must have the same shape and dtype")
        prec = _prop_dtype(S_light, "propagators")
        dev = self._torch_device()
        if not (S_light.is_cuda and S_strange.is_cuda) or S_light.device != dev:
            raise BBCError("correlate_noalloc takes device tensors on cuda:%d" % self.device)
        S_light, S_strange = S_light.contiguous(), S_strange.contiguous()
        n_t, Lz, Ly, Lx = S_light.shape[:4]
        t_arr, nt2 = _i32(t_list)
        if nt2 != n_t:
            raise BBCError("t_list must have one entry per slice")
        ch_arr, n_ch = _i32(channels)
        lat, _ = _i32([Lx, Ly, Lz])
        _check_tensor(out, (n_t, n_ch, Lz, Ly, Lx, 16), S_light.dtype, "out", dev)
        if prec == F32:
            if scale is None:
                raise BBCError("scale is required in the FP32 form")
            _check_tensor(scale, (n_t, n_ch), torch.float64, "scale", dev)
        e_arr = None
        if energy is not None:
            e_vals = [float(e) for e in energy]
            if len(e_vals) != n_ch:
                raise BBCError("energy must have one entry per channel")
            e_arr = (ctypes.c_double * n_ch)(*e_vals)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        _check(self._lib.bbc_correlate_noalloc(
            self._ptr, lat, prec, ctypes.c_void_p(S_light.data_ptr()), ctypes.c_void_p(S_strange.data_ptr()),
            n_t, t_arr, int(t0), n_ch, ch_arr, int(spin), e_arr, ctypes.c_void_p(out.data_ptr()),
            ctypes.c_void_p(scale.data_ptr()) if prec == F32 else None, ctypes.c_void_p(stream.cuda_stream)))
        return (out, scale) if prec == F32 else out

    def correlate_cpt(self, S_light, S_strange, t0, taus, channels, sign=1, energy=None, out=None, scale=None,
                      stream=None):
        """Forward/backward (CPT) average R_ch(r, tau) (Sec. 6): half the sum of the upper
        components on slice (t0 + tau) mod Lt and sign times the lower components on slice
        (t0 - tau) mod Lt, both normalised by exp(E tau).

        S_*:   device tensors [Lt, Lz, Ly, Lx, 12, 12] holding every time slice,
               complex128 (FP64 form) or complex64 (FP32 form).
        Returns ``out`` [n_tau, n_ch, Lz, Ly, Lx, 16]; in the FP32 form also ``scale``
        [n_tau, n_ch] float64.  Stream-ordered on ``stream`` (default: torch's current stream).
        """
        import torch

        if S_light.shape != S_strange.shape or S_light.dtype != S_strange.dtype:
            raise BBCError("S_light and S_strange must have the same shape and dtype")
        prec = _prop_dtype(S_light, "propagators")
        if not (S_light.is_cuda and S_strange.is_cuda) or S_light.device != self._torch_device():
            raise BBCError("correlate_cpt takes device tensors on cuda:%d" % self.device)
        S_light = S_light.contiguous()
        S_strange = S_strange.contiguous()
        Lt, Lz, Ly, Lx = S_light.shape[:4]
        tau_arr, n_tau = _i32(taus)
        ch_arr, n_ch = _i32(channels)
        lat, _ = _i32([Lx, Ly, Lz])
        dev = S_light.device
        oshape = (n_tau, n_ch, Lz, Ly, Lx, 16)
        if out is None:
            out = torch.empty(oshape, dtype=S_light.dtype, device=dev)
        _check_tensor(out, oshape, S_light.dtype, "out", dev)
        if prec == F32:
            if scale is None:
                scale = torch.empty((n_tau, n_ch), dtype=torch.float64, device=dev)
            _check_tensor(scale, (n_tau, n_ch), torch.float64, "scale", dev)
        e_arr = None
        if energy is not None:
            e_vals = [float(e) for e in energy]
            if len(e_vals) != n_ch:
                raise BBCError("energy must have one entry per channel")
            e_arr = (ctypes.c_double * n_ch)(*e_vals)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        _check(self._lib.bbc_correlate_cpt(
            self._ptr, lat, int(Lt), prec, ctypes.c_void_p(S_light.data_ptr()),
            ctypes.c_void_p(S_strange.data_ptr()), int(t0), n_tau, tau_arr, n_ch, ch_arr, int(sign), e_arr,
            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(scale.data_ptr()) if prec == F32 else None,
            ctypes.c_void_p(stream.cuda_stream)))
        return (out, scale) if prec == F32 else out

    # ------------------------------------------------------- post-processing
    def _field_args(self, field, n_site_vals):
        import torch
        if not field.is_cuda:
            raise BBCError("post-processing fields must be device tensors")
        if field.dtype == torch.complex128:
            prec = F64
        elif field.dtype == torch.complex64:
            prec = F32
        else:
            raise BBCError("fields must be complex128 or complex64")
        if field.dim() < 4:
            raise BBCError("field must be [..., Lz, Ly, Lx, n]")
        Lz, Ly, Lx, n = field.shape[-4:]
        if n != n_site_vals:
            raise BBCError("last dimension must be %d" % n_site_vals)
        n_fields = field.numel() // (Lx * Ly * Lz * n)
        lat, _ = _i32([Lx, Ly, Lz])
        return prec, lat, n_fields, (Lz, Ly, Lx)

    def spin_project(self, C, W, out=None, stream=None):
        """out[..., m] = sum_s W[m, s] C[..., s] for C [..., Lz, Ly, Lx, 16] on the device;
        W: n_out x 16 complex (host, e.g. Clebsch-Gordan products)."""
        import numpy as np
        import torch
        C = C.contiguous()
        prec, lat, n_fields, sp = self._field_args(C, 16)
        Wn = np.ascontiguousarray(np.asarray(W, dtype=np.complex128))
        if Wn.ndim != 2 or Wn.shape[1] != 16:
            raise BBCError("W must be n_out x 16")
        n_out = Wn.shape[0]
        if out is None:
            out = torch.empty(C.shape[:-1] + (n_out,), dtype=C.dtype, device=C.device)
        _check_tensor(out, C.shape[:-1] + (n_out,), C.dtype, "out", C.device)
        w_arr = Wn.view(np.float64).ctypes.data_as(ctypes.c_void_p)
        if stream is None:
            stream = torch.cuda.current_stream(C.device)
        _check(self._lib.bbc_spin_project(self._ptr, lat, prec, n_fields, ctypes.c_void_p(C.data_ptr()), n_out,
                                          w_arr, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream.cuda_stream)))
        return out

    def cubic_project(self, F, complement=False, out=None, stream=None):
        """A1+ projection over the cubic group of F [..., L, L, L, n] (device); Q = 1 - P if complement."""
        import torch
        F = F.contiguous()
        prec, lat, n_fields, _ = self._field_args(F, F.shape[-1])
        if out is None:
            out = torch.empty_like(F)
        _check_tensor(out, F.shape, F.dtype, "out", F.device)
        if stream is None:
            stream = torch.cuda.current_stream(F.device)
        _check(self._lib.bbc_cubic_project(self._ptr, lat, prec, n_fields, F.shape[-1],
                                           ctypes.c_void_p(F.data_ptr()),
                                           CUBIC_A1_COMPLEMENT if complement else CUBIC_A1,
                                           ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream.cuda_stream)))
        return out

    def central_potential(self, R, inv_2mu, out=None, stream=None):
        """V(r, t) for the inner slices of R [..., n_t, Lz, Ly, Lx] complex128 on the device
        (leading dimensions: independent sequences, e.g. channels)."""
        import torch
        if not R.is_cuda or R.dtype != torch.complex128 or R.dim() < 4:
            raise BBCError("R must be a [..., n_t, Lz, Ly, Lx] complex128 device tensor")
        R = R.contiguous()
        n_t, Lz, Ly, Lx = R.shape[-4:]
        n_fields = R.numel() // (n_t * Lz * Ly * Lx) if R.numel() else 0
        lat, _ = _i32([Lx, Ly, Lz])
        oshape = R.shape[:-4] + (max(n_t - 2, 0), Lz, Ly, Lx)
        if out is None:
            out = torch.empty(oshape, dtype=R.dtype, device=R.device)
        _check_tensor(out, oshape, R.dtype, "out", R.device)
        if stream is None:
            stream = torch.cuda.current_stream(R.device)
        _check(self._lib.bbc_central_potential(self._ptr, lat, n_fields, n_t, ctypes.c_void_p(R.data_ptr()),
                                               float(inv_2mu), ctypes.c_void_p(out.data_ptr()),
                                               ctypes.c_void_p(stream.cuda_stream)))
        return out
