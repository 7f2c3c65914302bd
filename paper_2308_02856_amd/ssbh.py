"""Thin ctypes binding of libssbh.so (argument marshalling only).

Every step of the path runs in the library's HIP kernels; this module turns
torch tensors into device pointers and the current torch stream into a HIP
stream, and raises on error codes.  Bit strings are torch.int64 tensors that
hold the library's uint64 words bit for bit.  Importing this module fails
loudly when the library has not been built: there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
import re

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libssbh.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "ssbh.h")

OK, PENDING = 0, 1
E_INVAL, E_ABORT_OVERSIZE, E_NOMEM, E_DEVICE, E_UNKNOWN_JOB, E_UNSUPPORTED = (
    -1, -2, -3, -4, -5, -6)
E_PRECISION = -7
SAMPLE_IID, SAMPLE_PERMUTE, SAMPLE_EXPLICIT = 0, 1, 2
OUT_FIXED, OUT_RATIO, OUT_EXPLICIT = 0, 1, 2
K_AUTO, K_VALU, K_MFMA_I8, K_FFT, K_MFMA_F4 = 0, 1, 2, 3, 4

_STATUS_NAMES = {OK: "OK", PENDING: "PENDING", E_INVAL: "E_INVAL",
                 E_ABORT_OVERSIZE: "E_ABORT_OVERSIZE", E_NOMEM: "E_NOMEM",
                 E_DEVICE: "E_DEVICE", E_UNKNOWN_JOB: "E_UNKNOWN_JOB",
                 E_UNSUPPORTED: "E_UNSUPPORTED", E_PRECISION: "E_PRECISION"}

_lib = None
_vp, _u64, _u32, _i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32


class Job(ctypes.Structure):
    """ssbh_job (include/ssbh.h)."""
    _fields_ = [("inp", ctypes.c_void_p), ("in_on_device", ctypes.c_int),
                ("n_bits", ctypes.c_uint64), ("n_sub", ctypes.c_uint32),
                ("sample_key", ctypes.c_uint64), ("l_ub", ctypes.c_uint64),
                ("out_rule", ctypes.c_uint32), ("out_a", ctypes.c_uint64),
                ("out_b", ctypes.c_uint64), ("seed_key", ctypes.c_uint64),
                ("out", ctypes.c_void_p), ("out_on_device", ctypes.c_int)]


class Result(ctypes.Structure):
    """ssbh_result (include/ssbh.h)."""
    _fields_ = [("status", ctypes.c_int32), ("out_bits", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class PipelineDesc(ctypes.Structure):
    """ssbh_pipeline_desc (include/ssbh.h)."""
    _fields_ = [("d_in", ctypes.c_void_p), ("n_bits", ctypes.c_uint64),
                ("n_sub", ctypes.c_uint32), ("mode", ctypes.c_uint32),
                ("sample_key", ctypes.c_uint64), ("d_assign", ctypes.c_void_p),
                ("l_ub", ctypes.c_uint64), ("d_sub", ctypes.c_void_p),
                ("sub_capacity_words", ctypes.c_uint64),
                ("d_len", ctypes.c_void_p), ("d_word_off", ctypes.c_void_p),
                ("out_rule", ctypes.c_uint32), ("out_a", ctypes.c_uint64),
                ("out_b", ctypes.c_uint64), ("d_out_len", ctypes.c_void_p),
                ("d_seed", ctypes.c_void_p), ("seed_bits", ctypes.c_uint64),
                ("seed_stride", ctypes.c_uint64), ("m_cap", ctypes.c_uint64),
                ("kernel", ctypes.c_uint32), ("d_out", ctypes.c_void_p),
                ("out_capacity_bits", ctypes.c_uint64),
                ("d_out_total_bits", ctypes.c_void_p),
                ("d_status", ctypes.c_void_p), ("d_keep", ctypes.c_void_p)]


class SsbhError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def header_functions() -> list[str]:
    """Names of the functions that include/ssbh.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ssbh_[a-z0-9_]+)\s*\(", text)))


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    L.ssbh_last_error.restype = ctypes.c_char_p
    L.ssbh_last_error.argtypes = []
    L.ssbh_create.restype = _i32
    L.ssbh_create.argtypes = [ctypes.c_int, _u64, ctypes.POINTER(_vp)]
    L.ssbh_destroy.restype = None
    L.ssbh_destroy.argtypes = [_vp]
    L.ssbh_num_cus.restype = ctypes.c_int
    L.ssbh_num_cus.argtypes = [_vp]
    L.ssbh_sample.restype = _i32
    L.ssbh_sample.argtypes = [_vp, _vp, _u64, _u32, _u32, _u64, _vp, _u64,
                              _vp, _u64, _vp, _vp, _vp, _vp]
    L.ssbh_sample_sifted.restype = _i32
    L.ssbh_sample_sifted.argtypes = [_vp, _vp, _vp, _u64, _u32, _u32, _u64,
                                     _vp, _u64, _vp, _u64, _vp, _vp, _vp, _vp]
    L.ssbh_ub_threshold.restype = _i32
    L.ssbh_ub_threshold.argtypes = [_u64, ctypes.c_double, _u32,
                                    ctypes.c_double, ctypes.POINTER(_u64),
                                    ctypes.POINTER(ctypes.c_double)]
    L.ssbh_geat_key_length.restype = _i32
    L.ssbh_geat_key_length.argtypes = [ctypes.POINTER(GeatParams),
                                       ctypes.c_double, ctypes.c_double,
                                       ctypes.POINTER(ctypes.c_double)]
    L.ssbh_geat_optimise.restype = _i32
    L.ssbh_geat_optimise.argtypes = [ctypes.POINTER(GeatParams),
                                     ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
    L.ssbh_hash_batch.restype = _i32
    L.ssbh_hash_batch.argtypes = [_vp, _vp, _u64, _vp, _vp, _u32, _u32, _u64,
                                  _u64, _vp, _vp, _u64, _u64, _u64, _u32, _vp,
                                  _u64, _vp, _vp, _vp]
    L.ssbh_seed_from_key.restype = _i32
    L.ssbh_seed_from_key.argtypes = [_vp, _u64, _vp, _u64, _vp]
    L.ssbh_permutation.restype = _i32
    L.ssbh_hash_batch_noalloc.restype = _i32
    L.ssbh_hash_batch_noalloc.argtypes = L.ssbh_hash_batch.argtypes
    L.ssbh_permutation.argtypes = [_vp, _u64, _u64, _vp, _vp]
    L.ssbh_set_schedule.restype = _i32
    L.ssbh_set_schedule.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _u32, _u32]
    L.ssbh_pipeline_create.restype = _i32
    L.ssbh_pipeline_create.argtypes = [_vp, ctypes.POINTER(PipelineDesc),
                                       ctypes.POINTER(_vp)]
    L.ssbh_pipeline_launch.restype = _i32
    L.ssbh_pipeline_launch.argtypes = [_vp, _vp]
    L.ssbh_pipeline_destroy.restype = None
    L.ssbh_pipeline_destroy.argtypes = [_vp]
    L.ssbh_tune.restype = _i32
    L.ssbh_tune.argtypes = [_vp, _vp, _u64, _vp, _vp, _u32, _u32, _u64, _u64,
                            _vp, _vp, _u64, _u64, _u64, _vp, _u64, _vp, _vp,
                            _u32, ctypes.c_char_p, _u64, _vp]
    L.ssbh_tune_table.restype = _i32
    L.ssbh_tune_table.argtypes = [_vp, ctypes.c_char_p, _u64]
    L.ssbh_last_schedule.restype = _i32
    L.ssbh_last_schedule.argtypes = [_vp, ctypes.c_char_p, _u64]
    L.ssbh_set_mfma_schedule.restype = _i32
    L.ssbh_set_mfma_schedule.argtypes = [_vp, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int]
    L.ssbh_set_sample_path.restype = _i32
    L.ssbh_set_sample_path.argtypes = [_vp, ctypes.c_int]
    L.ssbh_set_timing.restype = _i32
    L.ssbh_set_timing.argtypes = [_vp, ctypes.c_int]
    L.ssbh_timing_report.restype = _i32
    L.ssbh_timing_report.argtypes = [_vp, ctypes.c_char_p, _u64]
    L.ssbh_set_fft_schedule.restype = _i32
    L.ssbh_set_fft_schedule.argtypes = [_vp, _u32]
    L.ssbh_set_fft_packing.restype = _i32
    L.ssbh_set_fft_packing.argtypes = [_vp, ctypes.c_int]
    L.ssbh_set_fft_storage.restype = _i32
    L.ssbh_set_fft_storage.argtypes = [_vp, ctypes.c_int]
    L.ssbh_set_column_path.restype = _i32
    L.ssbh_set_column_path.argtypes = [_vp, ctypes.c_int]
    L.ssbh_job_out_words.restype = _u64
    L.ssbh_job_out_words.argtypes = [ctypes.POINTER(Job)]
    L.ssbh_submit.restype = _i32
    L.ssbh_submit.argtypes = [_vp, ctypes.POINTER(Job), ctypes.POINTER(_u64)]
    L.ssbh_poll.restype = _i32
    L.ssbh_poll.argtypes = [_vp, _u64, ctypes.POINTER(Result)]
    L.ssbh_serve_counts.restype = _i32
    L.ssbh_serve_counts.argtypes = [_vp, ctypes.POINTER(_u64),
                                    ctypes.POINTER(_u64), ctypes.POINTER(_u64)]
    _lib = L
    return L


def _check(rc: int) -> int:
    if rc < 0:
        msg = lib().ssbh_last_error().decode(errors="replace")
        raise SsbhError(rc, msg)
    return rc


def _ptr(t) -> int | None:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    return t.data_ptr()


def _stream(stream) -> int | None:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def words(n_bits: int) -> int:
    return (int(n_bits) + 63) // 64


class Context:
    """A library context on one GPU."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        self.device = int(device)
        self._h = _vp()
        _check(lib().ssbh_create(self.device, int(hbm_budget),
                                 ctypes.byref(self._h)))
        self.num_cus = lib().ssbh_num_cus(self._h)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().ssbh_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self):
        return torch.device("cuda", self.device)

    # ------------------------------------------------------------ sampling

    def sample(self, inp, n_bits: int, n_sub: int, mode: int = SAMPLE_IID,
               key: int = 0, assign=None, l_ub: int = 0, sub=None,
               sub_capacity: int | None = None, length=None, word_off=None,
               status=None, stream=None):
        """ssbh_sample; returns (sub, len, word_off, status) device tensors."""
        dev = self._dev()
        if sub_capacity is None:
            if mode == SAMPLE_PERMUTE:
                sub_capacity = n_sub * words(n_bits // max(n_sub, 1))
            else:
                sub_capacity = words(n_bits) + n_sub
        if sub is None:
            sub = torch.empty(max(1, sub_capacity), dtype=torch.int64, device=dev)
        if length is None:
            length = torch.empty(max(1, n_sub), dtype=torch.int64, device=dev)
        if word_off is None:
            word_off = torch.empty(max(1, n_sub), dtype=torch.int64, device=dev)
        if status is None:
            status = torch.zeros(1, dtype=torch.int32, device=dev)
        _check(lib().ssbh_sample(self._h, _ptr(inp), int(n_bits), int(n_sub),
                                 int(mode), int(key) & (2**64 - 1),
                                 _ptr(assign), int(l_ub), _ptr(sub),
                                 int(sub_capacity), _ptr(length),
                                 _ptr(word_off), _ptr(status),
                                 _stream(stream)))
        return sub, length, word_off, status

    def sample_sifted(self, inp, keep, n_bits: int, n_sub: int,
                      mode: int = SAMPLE_IID, key: int = 0, assign=None,
                      l_ub: int = 0, sub=None, sub_capacity: int | None = None,
                      length=None, word_off=None, status=None, stream=None):
        """ssbh_sample_sifted; returns (sub, len, word_off, status)."""
        dev = self._dev()
        if sub_capacity is None:
            sub_capacity = words(n_bits) + n_sub
        if sub is None:
            sub = torch.empty(max(1, sub_capacity), dtype=torch.int64, device=dev)
        if length is None:
            length = torch.empty(max(1, n_sub), dtype=torch.int64, device=dev)
        if word_off is None:
            word_off = torch.empty(max(1, n_sub), dtype=torch.int64, device=dev)
        if status is None:
            status = torch.zeros(1, dtype=torch.int32, device=dev)
        _check(lib().ssbh_sample_sifted(
            self._h, _ptr(inp), _ptr(keep), int(n_bits), int(n_sub), int(mode),
            int(key) & (2**64 - 1), _ptr(assign), int(l_ub), _ptr(sub),
            int(sub_capacity), _ptr(length), _ptr(word_off), _ptr(status),
            _stream(stream)))
        return sub, length, word_off, status

    # ------------------------------------------------------------- hashing

    def hash_batch(self, sub, sub_capacity: int, length, word_off, n_sub: int,
                   seed, seed_bits: int, m_cap: int, out_rule: int = OUT_FIXED,
                   out_a: int = 0, out_b: int = 1, out_len=None,
                   seed_stride: int = 0, kernel: int = K_AUTO, out=None,
                   out_capacity_bits: int | None = None, total=None,
                   status=None, stream=None, reset_status: bool = True):
        """ssbh_hash_batch; returns (out, total_bits, status) device tensors."""
        dev = self._dev()
        if out_capacity_bits is None:
            if out_rule == OUT_FIXED:
                out_capacity_bits = int(out_a) * int(n_sub)
            elif out_rule == OUT_RATIO:
                out_capacity_bits = (64 * int(sub_capacity) * int(out_a)) // int(out_b)
            else:
                out_capacity_bits = int(out_len.sum().item())
        if out is None:
            out = torch.empty(max(1, words(out_capacity_bits)), dtype=torch.int64,
                              device=dev)
        if total is None:
            total = torch.zeros(1, dtype=torch.int64, device=dev)
        if status is None:
            status = torch.zeros(1, dtype=torch.int32, device=dev)
        elif reset_status:
            status.zero_()
        _check(lib().ssbh_hash_batch(
            self._h, _ptr(sub), int(sub_capacity), _ptr(length),
            _ptr(word_off), int(n_sub), int(out_rule), int(out_a), int(out_b),
            _ptr(out_len), _ptr(seed), int(seed_bits), int(seed_stride),
            int(m_cap), int(kernel), _ptr(out), int(out_capacity_bits),
            _ptr(total), _ptr(status), _stream(stream)))
        return out, total, status

    def hash_batch_noalloc(self, sub, sub_capacity: int, length, word_off,
                           n_sub: int, seed, seed_bits: int, m_cap: int,
                           out, out_capacity_bits: int, total, status,
                           out_rule: int = OUT_FIXED, out_a: int = 0,
                           out_b: int = 1, out_len=None, seed_stride: int = 0,
                           kernel: int = K_AUTO, stream=None):
        """ssbh_hash_batch_noalloc: every buffer is the caller's (the
        library allocates nothing)."""
        _check(lib().ssbh_hash_batch_noalloc(
            self._h, _ptr(sub), int(sub_capacity), _ptr(length),
            _ptr(word_off), int(n_sub), int(out_rule), int(out_a), int(out_b),
            _ptr(out_len), _ptr(seed), int(seed_bits), int(seed_stride),
            int(m_cap), int(kernel), _ptr(out), int(out_capacity_bits),
            _ptr(total), _ptr(status), _stream(stream)))
        return out, total, status

    def seed_from_key(self, key: int, seed_bits: int, out=None, stream=None):
        if out is None:
            out = torch.empty(max(1, words(seed_bits)), dtype=torch.int64,
                              device=self._dev())
        _check(lib().ssbh_seed_from_key(self._h, int(key) & (2**64 - 1),
                                        _ptr(out), int(seed_bits),
                                        _stream(stream)))
        return out

    def permutation(self, key: int, n: int, out=None, stream=None):
        """ssbh_permutation: the keyed permutation of 0..n-1 (int32 tensor
        holding uint32 values)."""
        if out is None:
            out = torch.empty(max(1, int(n)), dtype=torch.int32,
                              device=self._dev())
        _check(lib().ssbh_permutation(self._h, int(key) & (2**64 - 1), int(n),
                                      _ptr(out), _stream(stream)))
        return out

    def tune(self, sub, sub_capacity: int, length, word_off, n_sub: int,
             seed, seed_bits: int, m_cap: int, out_rule: int = OUT_FIXED,
             out_a: int = 0, out_b: int = 1, out_len=None, seed_stride: int = 0,
             out=None, out_capacity_bits: int | None = None, total=None,
             status=None, reps: int = 2, stream=None) -> str:
        """ssbh_tune on these arguments; returns the timing table."""
        dev = self._dev()
        if out_capacity_bits is None:
            out_capacity_bits = (int(out_a) * int(n_sub) if out_rule == OUT_FIXED
                                 else (64 * int(sub_capacity) * int(out_a)) // int(out_b))
        if out is None:
            out = torch.empty(max(1, words(out_capacity_bits)), dtype=torch.int64,
                              device=dev)
        if total is None:
            total = torch.zeros(1, dtype=torch.int64, device=dev)
        if status is None:
            status = torch.zeros(1, dtype=torch.int32, device=dev)
        buf = ctypes.create_string_buffer(4096)
        _check(lib().ssbh_tune(
            self._h, _ptr(sub), int(sub_capacity), _ptr(length), _ptr(word_off),
            int(n_sub), int(out_rule), int(out_a), int(out_b), _ptr(out_len),
            _ptr(seed), int(seed_bits), int(seed_stride), int(m_cap), _ptr(out),
            int(out_capacity_bits), _ptr(total), _ptr(status), int(reps), buf,
            4096, _stream(stream)))
        return buf.value.decode()

    def tune_table(self) -> str:
        buf = ctypes.create_string_buffer(8192)
        _check(lib().ssbh_tune_table(self._h, buf, 8192))
        return buf.value.decode()

    def last_schedule(self) -> str:
        """Kernel and schedule of the last synchronous hash launch."""
        buf = ctypes.create_string_buffer(64)
        _check(lib().ssbh_last_schedule(self._h, buf, 64))
        return buf.value.decode()

    def pipeline(self, **kw) -> "Pipeline":
        """A captured sample -> hash graph; keyword names as in ssbh_pipeline_desc
        (tensors for the d_* fields)."""
        return Pipeline(self, **kw)

    # ------------------------------------------------------------- serving

    def make_job(self, inp, n_bits: int, n_sub: int, sample_key: int,
                 seed_key: int, out_rule: int = OUT_RATIO, out_a: int = 2,
                 out_b: int = 5, l_ub: int = 0, out=None) -> tuple:
        """An ssbh_job over a device input; allocates the device output."""
        j = Job(inp=_ptr(inp), in_on_device=1, n_bits=int(n_bits),
                n_sub=int(n_sub), sample_key=int(sample_key) & (2**64 - 1),
                l_ub=int(l_ub), out_rule=int(out_rule), out_a=int(out_a),
                out_b=int(out_b), seed_key=int(seed_key) & (2**64 - 1),
                out=None, out_on_device=1)
        nw = int(lib().ssbh_job_out_words(ctypes.byref(j)))
        if out is None:
            out = torch.empty(max(1, nw), dtype=torch.int64, device=self._dev())
        j.out = _ptr(out)
        return j, out

    def submit(self, job: Job) -> int:
        """ssbh_submit: queue a job (its input must already be on the GPU)."""
        jid = _u64()
        _check(lib().ssbh_submit(self._h, ctypes.byref(job), ctypes.byref(jid)))
        return int(jid.value)

    def poll(self, job_id: int):
        """None while pending; else the Result (terminal status included)."""
        r = Result()
        rc = lib().ssbh_poll(self._h, int(job_id), ctypes.byref(r))
        if rc == PENDING:
            return None
        if rc == E_UNKNOWN_JOB or rc == E_INVAL:
            _check(rc)
        return r

    def serve_counts(self):
        p, r, f = _u64(), _u64(), _u64()
        _check(lib().ssbh_serve_counts(self._h, ctypes.byref(p),
                                       ctypes.byref(r), ctypes.byref(f)))
        return int(p.value), int(r.value), int(f.value)

    def set_schedule(self, r: int = 0, waves: int = 0, tile_cols: int = 0,
                     chunk_cols: int = 0):
        """Force the VALU schedule (0 = library choice); bits do not change."""
        _check(lib().ssbh_set_schedule(self._h, int(r), int(waves),
                                       int(tile_cols), int(chunk_cols)))

    def set_mfma_schedule(self, mt: int = 0, nt: int = 0, wm: int = 0,
                          ksplit: int = 0):
        """Force the matrix-core schedule (0s = library choice)."""
        _check(lib().ssbh_set_mfma_schedule(self._h, int(mt), int(nt), int(wm),
                                            int(ksplit)))

    def set_sample_path(self, path: int = 0):
        """Placement kernels of the sampling: 0 = library choice, 1 = one
        wavefront per segment / the direct permutation gather."""
        _check(lib().ssbh_set_sample_path(self._h, int(path)))

    def set_timing(self, on: bool = True):
        """Record HIP events around the main kernels of synchronous calls."""
        _check(lib().ssbh_set_timing(self._h, 1 if on else 0))

    def timing_report(self) -> dict:
        """{kernel: (launches, total_ms)} since the last report."""
        buf = ctypes.create_string_buffer(4096)
        _check(lib().ssbh_timing_report(self._h, buf, 4096))
        out = {}
        for line in buf.value.decode().splitlines():
            name, cnt, ms = line.split()
            out[name] = (int(cnt), float(ms))
        return out

    def set_fft_schedule(self, chunk_pairs: int = 0):
        """Force the FFT hash's chunk of transforms (0 = library)."""
        _check(lib().ssbh_set_fft_schedule(self._h, int(chunk_pairs)))

    def set_fft_packing(self, per_part: int = 0):
        """Sub-blocks per transform part: 1, 2 (x_lo + 2^18 x_hi) or 0 =
        library choice."""
        _check(lib().ssbh_set_fft_packing(self._h, int(per_part)))

    def set_fft_storage(self, bits: int = 0):
        """FFT transform data between passes: 64 (doubles), 32 (floats) or
        0 = library choice."""
        _check(lib().ssbh_set_fft_storage(self._h, int(bits)))

    def set_column_path(self, scalar_x: int = -1):
        """Column words via LDS (0), scalar loads (1) or library choice (-1)."""
        _check(lib().ssbh_set_column_path(self._h, int(scalar_x)))


class Pipeline:
    """ssbh_pipeline: the hot path captured into a HIP graph."""

    def __init__(self, ctx: Context, **kw):
        self.ctx = ctx
        self._keep = dict(kw)          # tensors must outlive the graph
        d = PipelineDesc()
        for name, _ in PipelineDesc._fields_:
            if name not in kw:
                continue
            v = kw[name]
            if isinstance(v, torch.Tensor):
                setattr(d, name, _ptr(v))
            else:
                setattr(d, name, v)
        self._h = _vp()
        _check(lib().ssbh_pipeline_create(ctx.handle, ctypes.byref(d),
                                          ctypes.byref(self._h)))

    def launch(self, stream=None):
        _check(lib().ssbh_pipeline_launch(self._h, _stream(stream)))

    def close(self):
        if self._h:
            lib().ssbh_pipeline_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ub_threshold(n_rounds: int, p_sift: float, n_sub: int,
                 eps: float) -> tuple[int, float]:
    """ssbh_ub_threshold: (L_S^UB, abort-chance bound at it)."""
    l_ub = _u64()
    at = ctypes.c_double()
    _check(lib().ssbh_ub_threshold(int(n_rounds), float(p_sift), int(n_sub),
                                   float(eps), ctypes.byref(l_ub),
                                   ctypes.byref(at)))
    return int(l_ub.value), float(at.value)


class GeatParams(ctypes.Structure):
    """ssbh_geat_params."""
    _fields_ = [(k, ctypes.c_double) for k in (
        "n_rounds", "p_x", "q_tol", "eta_tol", "e_bit", "f_ec", "eps_sec",
        "eps_sm", "p_omega", "d_x", "eps_abort")] + [("n_sub", ctypes.c_uint32)]


def _geat_params(params: dict) -> GeatParams:
    return GeatParams(**{k: params[k] for k, _ in GeatParams._fields_})


def geat_key_length(params: dict, alpha: float, e_tangent: float) -> float:
    """ssbh_geat_key_length: total key length (bits) at fixed alpha, e_t."""
    out = ctypes.c_double()
    p = _geat_params(params)
    _check(lib().ssbh_geat_key_length(ctypes.byref(p), float(alpha),
                                      float(e_tangent), ctypes.byref(out)))
    return float(out.value)


def geat_optimise(params: dict) -> tuple[float, float, float]:
    """ssbh_geat_optimise: (key length, alpha, e_tangent) at the maximum."""
    kb, a, e = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    p = _geat_params(params)
    _check(lib().ssbh_geat_optimise(ctypes.byref(p), ctypes.byref(kb),
                                    ctypes.byref(a), ctypes.byref(e)))
    return float(kb.value), float(a.value), float(e.value)


def status_name(code: int) -> str:
    return _STATUS_NAMES.get(int(code), str(code))
