"""ctypes binding of ``libpcmm.so`` (argument marshalling only).

Every computation runs in the HIP library; this module converts torch device
tensors and numpy host arrays into the C ABI of ``include/pcmm.h`` and
``include/pcmm_diag.h`` and back.  Loading fails loudly if the library has not
been built (``python -m paper_2504_14497_amd.build``): there is no fallback.

Device point matrices are int32 torch tensors of shape (npts * form * 8, ld)
holding 32-bit limbs (see ``pcmm.h``); ``points_to_soa``/``soa_to_points``
convert to and from the 64-byte big-endian (x || y) host format.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcmm.so")

AFFINE = 2
JACOBIAN = 3
STAGE_EVENTS = 6  # PCMM_STAGE_EVENTS

_STATUS = {0: "PCMM_OK", -1: "PCMM_EINVAL", -2: "PCMM_ERANGE", -3: "PCMM_ENOMEM",
           -4: "PCMM_EDEVICE", -5: "PCMM_ENOTONCURVE", -6: "PCMM_ETOOLARGE"}
STATIC_SCRATCH_BYTES = 64 << 20  # PCMM_STATIC_SCRATCH_BYTES


class PCMMError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {_STATUS.get(code, code)}")
        self.code = code


class Mat(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("cols", ctypes.c_int32), ("npts", ctypes.c_int32),
                ("form", ctypes.c_int32), ("ld", ctypes.c_int64), ("d", ctypes.c_void_p)]


class PointBE(ctypes.Structure):
    _fields_ = [("x", ctypes.c_uint8 * 32), ("y", ctypes.c_uint8 * 32)]


class CussenCfg(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("group", ctypes.c_int32), ("k_split", ctypes.c_int32),
                ("k_chunk", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("stage_events", ctypes.POINTER(ctypes.c_void_p))]


def cussen_cfg(rounds=4, group=0, k_split=0, k_chunk=0, profile=0, stage_events=None) -> CussenCfg:
    """A pcmm_cussen_cfg.  stage_events: None or PCMM_STAGE_EVENTS torch.cuda
    Events (timing enabled, each recorded once beforehand so that its HIP
    handle exists) that the call records its stage boundaries into."""
    cfg = CussenCfg(rounds, group, k_split, k_chunk, profile, None)
    if stage_events is not None:
        if len(stage_events) != STAGE_EVENTS:
            raise ValueError(f"need {STAGE_EVENTS} events")
        arr = (ctypes.c_void_p * STAGE_EVENTS)(*[int(e.cuda_event) for e in stage_events])
        if not all(arr):
            raise ValueError("record each event once before handing it over")
        cfg.stage_events = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
        cfg._keep = (arr, tuple(stage_events))
    return cfg


class CussenStats(ctypes.Structure):
    _fields_ = [("level_mults", ctypes.c_int64), ("level_adds", ctypes.c_int64),
                ("table_entries", ctypes.c_int64), ("table_adds", ctypes.c_int64),
                ("accum_adds", ctypes.c_int64), ("max_entries", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64),
                ("combo_adds", ctypes.c_int64), ("digit_entries", ctypes.c_int64),
                ("k_split", ctypes.c_int32), ("lanes_per_chain", ctypes.c_int32),
                ("group", ctypes.c_int32), ("coop_lanes", ctypes.c_int32),
                ("ms_upload", ctypes.c_float), ("ms_table", ctypes.c_float),
                ("ms_accumulate", ctypes.c_float), ("ms_reduce", ctypes.c_float),
                ("ms_normalize", ctypes.c_float), ("ms_total", ctypes.c_float)]

    def as_dict(self):
        return {k: (float(getattr(self, k)) if k.startswith("ms_") else int(getattr(self, k)))
                for k, _ in self._fields_}


class StrassenCfg(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class StrassenStats(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("leaf_bits", ctypes.c_int32), ("leaves", ctypes.c_int64),
                ("block_adds", ctypes.c_int64), ("leaf_ladder_ops", ctypes.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


GROUP_AUTO = -1          # PCMM_GROUP_AUTO
PLAN_MAX_PROBLEMS = 64   # PCMM_PLAN_MAX_PROBLEMS


class Problem(ctypes.Structure):
    """pcmm_problem"""
    _fields_ = [("A", ctypes.c_void_p), ("m", ctypes.c_int32), ("n", ctypes.c_int32), ("l", ctypes.c_int32),
                ("bits", ctypes.c_int32), ("is_signed", ctypes.c_int32), ("c_form", ctypes.c_int32),
                ("cfg", CussenCfg)]


_lib = None

# symbol -> (argtypes, restype)
_VP = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SIG = {
    "pcmm_keygen": ([ctypes.c_uint64, _VP, ctypes.POINTER(PointBE)], _I32),
    "pcmm_encrypt": ([ctypes.POINTER(PointBE), _VP, _I32, _I32, ctypes.c_uint64, _I64,
                      ctypes.POINTER(Mat), _VP, ctypes.c_size_t, _VP], _I32),
    "pcmm_encrypt_workspace": ([], ctypes.c_size_t),
    "pcmm_schoolbook": ([_VP, _I32, _I32, _I32, _I32, ctypes.POINTER(Mat), ctypes.POINTER(Mat), _VP,
                         ctypes.c_size_t, _VP], _I32),
    "pcmm_schoolbook_workspace": ([_I32, _I32, _I32, _I32], ctypes.c_size_t),
    "pcmm_cussen": ([_VP, _I32, _I32, _I32, _I32, ctypes.POINTER(Mat), ctypes.POINTER(Mat),
                     ctypes.POINTER(CussenCfg), _VP, ctypes.c_size_t, ctypes.POINTER(CussenStats),
                     _VP], _I32),
    "pcmm_cussen_static": ([_VP, _I32, _I32, _I32, _I32, ctypes.POINTER(Mat), ctypes.POINTER(Mat),
                            ctypes.POINTER(CussenCfg), ctypes.POINTER(CussenStats), _VP], _I32),
    "pcmm_cussen_workspace": ([_VP, _I32, _I32, _I32, _I32, _I32, _I32, ctypes.POINTER(CussenCfg),
                               ctypes.POINTER(ctypes.c_size_t)], _I32),
    "pcmm_cussen_plan_stats": ([_VP, _I32, _I32, _I32, _I32, ctypes.POINTER(CussenCfg),
                                ctypes.POINTER(CussenStats)], _I32),
    "pcmm_plan_create": ([ctypes.POINTER(Problem), _I32, ctypes.POINTER(_VP)], _I32),
    "pcmm_plan_destroy": ([_VP], _I32),
    "pcmm_plan_workspace": ([_VP, ctypes.POINTER(ctypes.c_size_t)], _I32),
    "pcmm_plan_stats": ([_VP, _I32, ctypes.POINTER(CussenStats)], _I32),
    "pcmm_plan_run": ([_VP, ctypes.POINTER(Mat), ctypes.POINTER(Mat), _VP, ctypes.c_size_t,
                       ctypes.POINTER(_VP), _VP], _I32),
    "pcmm_plan_resident_bytes": ([_VP, ctypes.POINTER(ctypes.c_size_t)], _I32),
    "pcmm_plan_make_resident": ([_VP, _VP, ctypes.c_size_t, _VP], _I32),
    "pcmm_plan_selected_workspace": ([_VP, ctypes.POINTER(_I32), _I32, ctypes.POINTER(ctypes.c_size_t)], _I32),
    "pcmm_plan_run_selected": ([_VP, ctypes.POINTER(_I32), _I32, ctypes.POINTER(Mat), ctypes.POINTER(Mat), _VP,
                                ctypes.c_size_t, ctypes.POINTER(_VP), _VP], _I32),
    "pcmm_strassen": ([_VP, _I32, _I32, _I32, _I32, ctypes.POINTER(Mat), ctypes.POINTER(Mat),
                       ctypes.POINTER(StrassenCfg), _VP, ctypes.c_size_t, ctypes.POINTER(StrassenStats), _VP], _I32),
    "pcmm_strassen_workspace": ([_I32, _I32, _I32, _I32, ctypes.POINTER(StrassenCfg),
                                 ctypes.POINTER(ctypes.c_size_t)], _I32),
    "pcmm_dlog_table_bytes": ([_I32, ctypes.POINTER(ctypes.c_size_t)], _I32),
    "pcmm_dlog_table_workspace": ([_I32, ctypes.POINTER(ctypes.c_size_t)], _I32),
    "pcmm_dlog_table_build": ([_I32, _VP, ctypes.c_size_t, _VP, ctypes.c_size_t, _VP], _I32),
    "pcmm_decrypt_workspace": ([_I64, _I64, _I32, ctypes.POINTER(ctypes.c_size_t)], _I32),
    "pcmm_decrypt": ([_VP, ctypes.POINTER(Mat), _I64, _VP, ctypes.c_size_t, _I32, _VP, _VP, ctypes.c_size_t,
                      _VP], _I32),
    "pcmm_normalize": ([ctypes.POINTER(Mat), ctypes.POINTER(Mat), _VP, ctypes.c_size_t, _VP], _I32),
    "pcmm_normalize_workspace": ([_I64, _I32], ctypes.c_size_t),
    "pcmm_decrypt_to_points": ([_VP, ctypes.POINTER(Mat), ctypes.POINTER(Mat), _VP], _I32),
    "pcmm_strerror": ([_I32], ctypes.c_char_p),
    "pcmm_diag_field": ([_I32, _VP, _VP, _VP, _I64, _VP], _I32),
    "pcmm_diag_point": ([_I32, ctypes.POINTER(Mat), ctypes.POINTER(Mat), _VP, _I32,
                         ctypes.POINTER(Mat), _VP], _I32),
    "pcmm_diag_probe": ([_I32, _I64, _I32, ctypes.POINTER(ctypes.c_double),
                         ctypes.POINTER(ctypes.c_double)], _I32),
    "pcmm_diag_device": ([ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I64),
                          ctypes.c_char_p], _I32),
    "pcmm_diag_copy": ([_VP, _VP, _I64, _VP], _I32),
    "pcmm_diag_field_raw": ([_I32, _VP, _VP, _VP, _I64, _VP], _I32),
    "pcmm_diag_plan_check": ([_VP, _I32, _I32, _I32, _I32, _I32, _I32, ctypes.POINTER(_I32)], _I32),
    "pcmm_paillier_create": ([_VP, ctypes.POINTER(_VP)], _I32),
    "pcmm_paillier_destroy": ([_VP], _I32),
    "pcmm_paillier_encrypt": ([_VP, _VP, _I64, ctypes.c_uint64, _I64, _VP, _VP], _I32),
    "pcmm_paillier_schoolbook_workspace": ([_I32, _I32, _I32, ctypes.POINTER(ctypes.c_size_t)], _I32),
    "pcmm_paillier_schoolbook": ([_VP, _VP, _I32, _I32, _I32, _I32, _VP, _VP, _VP, ctypes.c_size_t, _VP], _I32),
    "pcmm_paillier_cussen_workspace": ([_VP, _I32, _I32, _I32, _I32, ctypes.POINTER(CussenCfg),
                                        ctypes.POINTER(ctypes.c_size_t)], _I32),
    "pcmm_paillier_cussen": ([_VP, _VP, _I32, _I32, _I32, _I32, _VP, _VP, ctypes.POINTER(CussenCfg), _VP,
                              ctypes.c_size_t, ctypes.POINTER(CussenStats), _VP], _I32),
    "pcmm_paillier_diag": ([_VP, _I32, _VP, _VP, _VP, _I64, _VP], _I32),
    "pcmm_paillier_diag_constants": ([_VP, _VP, _VP, _VP, _VP], _I32),
}

EXPORTED = tuple(_SIG)


def lib():
    """Load libpcmm.so (no fallback: raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch brings its own HIP runtime (libamdhip64.so, soname
        # libamdhip64.so.7).  Loaded first, it is the runtime that
        # libpcmm.so's dependency resolves to; loaded after libpcmm.so, it
        # would be a second runtime in the process, and whichever initialised
        # second finds no device.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libpcmm.so not found at {LIB_PATH}; build it with "
                               "`python -m paper_2504_14497_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIG.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _call(name, *args):
    rc = getattr(lib(), name)(*args)
    if rc != 0:
        raise PCMMError(rc, name)


# ---------------------------------------------------------------- layout helpers

def ints_to_limbs(vals) -> np.ndarray:
    """Python ints (< 2^256) -> uint32 array (8, count), limb-major."""
    vals = list(vals)
    out = np.zeros((8, len(vals)), dtype=np.uint32)
    for e, v in enumerate(vals):
        for w in range(8):
            out[w, e] = (v >> (32 * w)) & 0xFFFFFFFF
    return out


def limbs_to_ints(arr) -> list:
    a = np.asarray(arr, dtype=np.uint64)
    return [sum(int(a[w, e]) << (32 * w) for w in range(8)) for e in range(a.shape[1])]


def be_to_limbs(be: np.ndarray) -> np.ndarray:
    """(count, 32) big-endian bytes -> (8, count) little-endian 32-bit limbs."""
    be = np.ascontiguousarray(be, dtype=np.uint8).reshape(-1, 32)
    words = be.view(">u4").astype(np.uint32)  # (count, 8), most significant first
    return np.ascontiguousarray(words[:, ::-1].T)


def limbs_to_be(limbs: np.ndarray) -> np.ndarray:
    """(8, count) limbs -> (count, 32) big-endian bytes."""
    w = np.ascontiguousarray(np.asarray(limbs, dtype=np.uint32).T[:, ::-1]).astype(">u4")
    return w.view(np.uint8).reshape(-1, 32)


def points_to_soa(pts: np.ndarray, npts: int) -> np.ndarray:
    """(count, 64 * npts) host points (x || y big-endian, per point) ->
    (npts * 2 * 8, count) uint32 planes of an affine device matrix."""
    pts = np.ascontiguousarray(pts, dtype=np.uint8).reshape(-1, 64 * npts)
    count = pts.shape[0]
    planes = np.zeros((npts * 2 * 8, count), dtype=np.uint32)
    for pt in range(npts):
        for c in range(2):
            off = pt * 64 + c * 32
            planes[(pt * 2 + c) * 8:(pt * 2 + c + 1) * 8] = be_to_limbs(pts[:, off:off + 32])
    return planes


def soa_to_points(planes: np.ndarray, npts: int, count: int) -> np.ndarray:
    """Inverse of points_to_soa (affine planes) -> (count, 64 * npts) bytes."""
    planes = np.asarray(planes, dtype=np.uint32)
    out = np.zeros((count, 64 * npts), dtype=np.uint8)
    for pt in range(npts):
        for c in range(2):
            off = pt * 64 + c * 32
            out[:, off:off + 32] = limbs_to_be(planes[(pt * 2 + c) * 8:(pt * 2 + c + 1) * 8, :count])
    return out


def _tensor_ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def new_mat(rows, cols, npts, form, device="cuda", ld=None):
    """Allocate a device point matrix (torch int32 planes) and its descriptor."""
    import torch
    n = rows * cols
    if ld is None:
        ld = max(64, (n + 63) // 64 * 64)
    t = torch.zeros((npts * form * 8, ld), dtype=torch.int32, device=device)
    return t, mat_of(t, rows, cols, npts, form)


def mat_of(t, rows, cols, npts, form):
    assert t.dim() == 2 and t.shape[0] == npts * form * 8 and t.is_contiguous()
    return Mat(rows, cols, npts, form, t.shape[1], t.data_ptr())


def upload_points(pts: np.ndarray, rows, cols, npts, device="cuda"):
    """Host points (rows*cols, 64*npts) -> affine device matrix (tensor, Mat)."""
    import torch
    planes = points_to_soa(pts, npts)
    t, m = new_mat(rows, cols, npts, AFFINE, device=device)
    t[:, :planes.shape[1]] = torch.from_numpy(planes.view(np.int32)).to(device)
    return t, m


def download_points(t, rows, cols, npts) -> np.ndarray:
    """Affine device matrix -> host points (rows*cols, 64*npts) bytes."""
    planes = t.detach().cpu().numpy().view(np.uint32)
    return soa_to_points(planes, npts, rows * cols)


def stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------- diagnostics

def diag_field(op: int, a, b=None, stream=None):
    """Field op on Python ints via the device (returns Python ints)."""
    import torch
    a = list(a)
    n = len(a)
    ta = torch.from_numpy(ints_to_limbs(a).view(np.int32)).cuda().contiguous()
    tb = torch.from_numpy(ints_to_limbs(b if b is not None else [0] * n).view(np.int32)).cuda()
    to = torch.zeros_like(ta)
    _call("pcmm_diag_field", op, _tensor_ptr(ta), _tensor_ptr(tb), _tensor_ptr(to), n,
          stream_ptr(stream))
    torch.cuda.synchronize()
    return limbs_to_ints(to.cpu().numpy().view(np.uint32))


LIMB_BITS, NLIMBS = 29, 9


def diag_field_raw(op: int, a_limbs: np.ndarray, b_limbs: np.ndarray = None, stream=None) -> np.ndarray:
    """Raw-limb field op on (count, 9) int64/uint32 limb arrays; returns (count, 9) uint32."""
    import torch
    a = np.ascontiguousarray(np.asarray(a_limbs, dtype=np.int64).astype(np.uint32).T)
    b = a if b_limbs is None else np.ascontiguousarray(np.asarray(b_limbs, dtype=np.int64).astype(np.uint32).T)
    n = a.shape[1]
    ta = torch.from_numpy(a.view(np.int32)).cuda().contiguous()
    tb = torch.from_numpy(b.view(np.int32)).cuda().contiguous()
    to = torch.zeros_like(ta)
    _call("pcmm_diag_field_raw", op, _tensor_ptr(ta), _tensor_ptr(tb), _tensor_ptr(to), n, stream_ptr(stream))
    torch.cuda.synchronize()
    return np.ascontiguousarray(to.cpu().numpy().view(np.uint32).T)


def diag_point(op: int, P: np.ndarray, Q: np.ndarray = None, k=None, t: int = 0, stream=None):
    """Element-wise point op; P, Q: (count, 64) host points.  Returns the
    Jacobian result as a list of (X, Y, Z) canonical Python ints."""
    import torch
    count = P.shape[0]
    tp, mp = upload_points(P, 1, count, 1)
    if Q is not None:
        tq, mq = upload_points(Q, 1, count, 1)
        mq_ref = ctypes.byref(mq)
    else:
        mq_ref = None
    tr, mr = new_mat(1, count, 1, JACOBIAN)
    kt = None
    if k is not None:
        kt = torch.from_numpy(np.asarray(k, dtype=np.uint32).view(np.int32)).cuda()
    _call("pcmm_diag_point", op, ctypes.byref(mp), mq_ref,
          _tensor_ptr(kt) if kt is not None else None, t, ctypes.byref(mr), stream_ptr(stream))
    torch.cuda.synchronize()
    planes = tr.cpu().numpy().view(np.uint32)
    X = limbs_to_ints(planes[0:8, :count])
    Y = limbs_to_ints(planes[8:16, :count])
    Z = limbs_to_ints(planes[16:24, :count])
    return list(zip(X, Y, Z))


def diag_plan_check(A, bits: int, rounds: int = 4, group: int = 1) -> int:
    """Host-only symbolic check of the compression plan (0 = sound)."""
    A, signed = _host_A(A, bits)
    m, n = A.shape
    r = _I32(-1)
    _call("pcmm_diag_plan_check", A.ctypes.data_as(_VP), m, n, bits, signed, rounds, group, ctypes.byref(r))
    return r.value


def diag_probe(kind: int, iters: int, blocks: int):
    s = ctypes.c_double()
    o = ctypes.c_double()
    _call("pcmm_diag_probe", kind, iters, blocks, ctypes.byref(s), ctypes.byref(o))
    return s.value, o.value


def diag_copy(src, dst, stream=None):
    """Copy device tensor src into dst (same number of bytes, multiple of 16)."""
    assert src.numel() * src.element_size() == dst.numel() * dst.element_size()
    _call("pcmm_diag_copy", _tensor_ptr(src), _tensor_ptr(dst), src.numel() * src.element_size() // 4,
          stream_ptr(stream))


def device_info():
    cus = ctypes.c_int32()
    clk = ctypes.c_int32()
    lds = ctypes.c_int64()
    name = ctypes.create_string_buffer(64)
    _call("pcmm_diag_device", ctypes.byref(cus), ctypes.byref(clk), ctypes.byref(lds), name)
    return {"cus": cus.value, "clock_khz": clk.value, "lds_per_block": lds.value,
            "arch": name.value.decode()}


# ---------------------------------------------------------------- the C ABI, one call each

class DevPoints:
    """A device point matrix: torch int32 planes plus its pcmm_mat descriptor."""

    def __init__(self, t, rows, cols, npts, form):
        self.t = t
        self.rows, self.cols, self.npts, self.form = rows, cols, npts, form
        self.mat = mat_of(t, rows, cols, npts, form)

    @classmethod
    def empty(cls, rows, cols, npts, form, device="cuda"):
        t, _ = new_mat(rows, cols, npts, form, device=device)
        return cls(t, rows, cols, npts, form)

    @classmethod
    def from_host(cls, pts: np.ndarray, rows, cols, npts, device="cuda"):
        t, _ = upload_points(pts, rows, cols, npts, device=device)
        return cls(t, rows, cols, npts, AFFINE)

    def to_host(self) -> np.ndarray:
        """Affine matrix -> (rows, cols, 64 * npts) bytes."""
        assert self.form == AFFINE
        return download_points(self.t, self.rows, self.cols, self.npts).reshape(
            self.rows, self.cols, 64 * self.npts)

    def ref(self):
        return ctypes.byref(self.mat)


def _workspace(nbytes, device="cuda"):
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


_NARROW = {np.dtype(np.int16): np.int8, np.dtype(np.uint16): np.uint8}
_WIDE = {np.dtype(np.int8): np.int16, np.dtype(np.uint8): np.uint16}


def _host_A(A, bits: int):
    """A as the library reads it: signedness from the dtype (int8/int16
    signed, uint8/uint16 unsigned), element width from bits (1 byte up to 8
    bits, 2 bytes for 9..16)."""
    A = np.ascontiguousarray(A)
    if A.dtype not in (np.int8, np.uint8, np.int16, np.uint16):
        raise TypeError("A must be int8 / int16 (signed) or uint8 / uint16 (unsigned)")
    signed = 1 if A.dtype in (np.int8, np.int16) else 0
    if bits > 8 and A.dtype.itemsize == 1:
        A = A.astype(_WIDE[A.dtype])
    elif bits <= 8 and A.dtype.itemsize == 2:
        narrow = _NARROW[A.dtype]
        info = np.iinfo(narrow)
        if A.size and (A.min() < info.min or A.max() > info.max):
            raise PCMMError(-2, "plaintext entries outside the declared bit-width")
        A = A.astype(narrow)
    return A, signed


def keygen(seed: int):
    """(sk as 32 big-endian bytes, pk as 64 bytes x || y)."""
    sk = ctypes.create_string_buffer(32)
    pk = PointBE()
    _call("pcmm_keygen", seed, sk, ctypes.byref(pk))
    return sk.raw, bytes(pk.x) + bytes(pk.y)


def _point_be(pk: bytes) -> PointBE:
    p = PointBE()
    ctypes.memmove(p.x, pk[:32], 32)
    ctypes.memmove(p.y, pk[32:64], 32)
    return p


def encrypt(pk: bytes, msg, seed: int, idx0: int = 0, stream=None) -> DevPoints:
    """Encrypt a rows x cols int32 message matrix (host numpy or device tensor)."""
    import torch
    m = torch.as_tensor(msg, dtype=torch.int32).cuda().contiguous()
    rows, cols = m.shape
    out = DevPoints.empty(rows, cols, 2, AFFINE)
    ws = _workspace(lib().pcmm_encrypt_workspace())
    p = _point_be(pk)
    _call("pcmm_encrypt", ctypes.byref(p), _tensor_ptr(m), rows, cols, seed, idx0, out.ref(),
          _tensor_ptr(ws), ws.numel(), stream_ptr(stream))
    out._keep = (m, ws)
    return out


def schoolbook(A, bits: int, B: DevPoints, c_form: int = AFFINE, stream=None, workspace=None):
    A, signed = _host_A(A, bits)
    m, n = A.shape
    C = DevPoints.empty(m, B.cols, 2, c_form)
    need = lib().pcmm_schoolbook_workspace(m, n, B.cols, c_form)
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need)
    _call("pcmm_schoolbook", A.ctypes.data_as(_VP), m, n, bits, signed, B.ref(), C.ref(),
          _tensor_ptr(ws), ws.numel(), stream_ptr(stream))
    C._keep = (ws, A)  # the host copy of A is queued asynchronously
    return C


def strassen(A, bits: int, B: DevPoints, c_form: int = AFFINE, depth: int = 0, stream=None, workspace=None):
    """Strassen PC-MM (schoolbook leaves); returns (C, stats dict)."""
    A, signed = _host_A(A, bits)
    m, n = A.shape
    C = DevPoints.empty(m, B.cols, 2, c_form)
    cfg = StrassenCfg(depth, 0)
    need = ctypes.c_size_t()
    _call("pcmm_strassen_workspace", m, n, B.cols, c_form, ctypes.byref(cfg), ctypes.byref(need))
    ws = workspace if workspace is not None else _workspace(need.value)
    st = StrassenStats()
    _call("pcmm_strassen", A.ctypes.data_as(_VP), m, n, bits, signed, B.ref(), C.ref(), ctypes.byref(cfg),
          _tensor_ptr(ws), ws.numel(), ctypes.byref(st), stream_ptr(stream))
    C._keep = (ws, A)
    return C, st.as_dict()


def strassen_workspace_bytes(m: int, n: int, l: int, c_form: int = AFFINE, depth: int = 0) -> int:
    need = ctypes.c_size_t()
    _call("pcmm_strassen_workspace", m, n, l, c_form, ctypes.byref(StrassenCfg(depth, 0)), ctypes.byref(need))
    return need.value


def cussen_workspace_bytes(A, bits: int, l: int, c_form: int = AFFINE, cfg: CussenCfg = None) -> int:
    A, signed = _host_A(A, bits)
    m, n = A.shape
    nb = ctypes.c_size_t()
    _call("pcmm_cussen_workspace", A.ctypes.data_as(_VP), m, n, l, bits, signed, c_form,
          ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(nb))
    return nb.value


def cussen(A, bits: int, B: DevPoints, c_form: int = AFFINE, cfg: CussenCfg = None, stream=None,
           workspace=None, out: DevPoints = None):
    """Cussen PC-MM; returns (C, stats dict)."""
    A, signed = _host_A(A, bits)
    m, n = A.shape
    C = out if out is not None else DevPoints.empty(m, B.cols, 2, c_form)
    if workspace is not None:
        ws = workspace  # the library rejects one that is too small (PCMM_ENOMEM)
    else:
        ws = _workspace(cussen_workspace_bytes(A, bits, B.cols, C.form, cfg))
    st = CussenStats()
    _call("pcmm_cussen", A.ctypes.data_as(_VP), m, n, bits, signed, B.ref(), C.ref(),
          ctypes.byref(cfg) if cfg is not None else None, _tensor_ptr(ws), ws.numel(),
          ctypes.byref(st), stream_ptr(stream))
    C._keep = (ws,)
    return C, st.as_dict()


def cussen_static(A, bits: int, B: DevPoints, c_form: int = AFFINE, cfg: CussenCfg = None, stream=None,
                  out: DevPoints = None):
    """Cussen PC-MM through pcmm_cussen_static (workspace in the library's
    static device array, no allocation by the library); returns (C, stats)."""
    A, signed = _host_A(A, bits)
    m, n = A.shape
    C = out if out is not None else DevPoints.empty(m, B.cols, 2, c_form)
    st = CussenStats()
    _call("pcmm_cussen_static", A.ctypes.data_as(_VP), m, n, bits, signed, B.ref(), C.ref(),
          ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(st), stream_ptr(stream))
    return C, st.as_dict()


def cussen_plan_stats(A, bits: int, cfg: CussenCfg = None) -> dict:
    """Operation counts of the compression plan (host only, no GPU work)."""
    A, signed = _host_A(A, bits)
    m, n = A.shape
    st = CussenStats()
    _call("pcmm_cussen_plan_stats", A.ctypes.data_as(_VP), m, n, bits, signed,
          ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(st))
    return st.as_dict()


def normalize(C: DevPoints, stream=None, inplace=False) -> DevPoints:
    """Jacobian -> canonical affine."""
    assert C.form == JACOBIAN
    if inplace:
        # affine result in the first npts * 16 planes of the same buffer
        out = DevPoints.__new__(DevPoints)
        out.t = C.t
        out.rows, out.cols, out.npts, out.form = C.rows, C.cols, C.npts, AFFINE
        out.mat = Mat(C.rows, C.cols, C.npts, AFFINE, C.t.shape[1], C.t.data_ptr())
    else:
        out = DevPoints.empty(C.rows, C.cols, C.npts, AFFINE)
    ws = _workspace(lib().pcmm_normalize_workspace(C.rows * C.cols, C.npts))
    _call("pcmm_normalize", C.ref(), out.ref(), _tensor_ptr(ws), ws.numel(), stream_ptr(stream))
    out._keep = (ws,)
    return out


def decrypt_to_points(sk: bytes, C: DevPoints, stream=None) -> DevPoints:
    M = DevPoints.empty(C.rows, C.cols, 1, AFFINE)
    _call("pcmm_decrypt_to_points", sk, C.ref(), M.ref(), stream_ptr(stream))
    return M


def strerror(code: int) -> str:
    return lib().pcmm_strerror(code).decode()


class Plan:
    """A compiled pcmm_plan of one or more Cussen PC-MMs (pcmm_plan_*).

    problems: sequence of (A, bits, l, c_form, cfg) with A a host m x n
    int8 / int16 (signed) or uint8 / uint16 (unsigned) matrix and cfg a
    CussenCfg or None."""

    def __init__(self, problems):
        arr = (Problem * len(problems))()
        keep = []  # converted copies of A stay alive until pcmm_plan_create returns
        self.shapes = []
        for k, (A, bits, l, c_form, cfg) in enumerate(problems):
            A, signed = _host_A(A, bits)
            keep.append(A)
            m, n = A.shape
            arr[k] = Problem(A.ctypes.data, m, n, l, bits, signed, c_form,
                             cfg if cfg is not None else CussenCfg(4, 0, 0, 0, 0, None))
            self.shapes.append((m, n, l, c_form))
        h = ctypes.c_void_p()
        _call("pcmm_plan_create", arr, len(problems), ctypes.byref(h))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().pcmm_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self) -> int:
        n = ctypes.c_size_t()
        _call("pcmm_plan_workspace", self.h, ctypes.byref(n))
        return n.value

    def stats(self, index: int) -> dict:
        st = CussenStats()
        _call("pcmm_plan_stats", self.h, index, ctypes.byref(st))
        return st.as_dict()

    def outputs(self):
        return [DevPoints.empty(m, l, 2, c_form) for (m, n, l, c_form) in self.shapes]

    def run(self, B, C=None, workspace=None, stage_events=None, stream=None):
        """B: list of DevPoints (n_i x l_i ciphertexts); C: list of DevPoints
        or None (allocated).  Queues the run; returns C."""
        if C is None:
            C = self.outputs()
        if len(B) != len(self.shapes) or len(C) != len(self.shapes):
            raise ValueError("one B and one C per problem")
        Bm = (Mat * len(B))(*[b.mat for b in B])
        Cm = (Mat * len(C))(*[c.mat for c in C])
        ws = workspace if workspace is not None else _workspace(self.workspace_bytes())
        evp = None
        if stage_events is not None:
            if len(stage_events) != STAGE_EVENTS:
                raise ValueError(f"need {STAGE_EVENTS} events")
            evp = (ctypes.c_void_p * STAGE_EVENTS)(*[int(e.cuda_event) for e in stage_events])
        _call("pcmm_plan_run", self.h, Bm, Cm, _tensor_ptr(ws), ws.numel(), evp, stream_ptr(stream))
        for c in C:
            c._keep = (ws,)
        return C

    # resident plans and selected runs (serving)
    def make_resident(self, stream=None):
        """Copies the compiled arrays to a device buffer kept by this object."""
        import torch
        n = ctypes.c_size_t()
        _call("pcmm_plan_resident_bytes", self.h, ctypes.byref(n))
        self.resident = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        _call("pcmm_plan_make_resident", self.h, _tensor_ptr(self.resident), n.value, stream_ptr(stream))

    def selected_workspace_bytes(self, which) -> int:
        w = (ctypes.c_int32 * len(which))(*which)
        n = ctypes.c_size_t()
        _call("pcmm_plan_selected_workspace", self.h, w, len(which), ctypes.byref(n))
        return n.value

    def run_selected(self, which, B, C, workspace, stage_events=None, stream=None):
        """Runs problems `which` (repeats allowed) on B[r] -> C[r]; queues and returns."""
        if len(B) != len(which) or len(C) != len(which):
            raise ValueError("one B and one C per selected problem")
        w = (ctypes.c_int32 * len(which))(*which)
        Bm = (Mat * len(B))(*[b.mat for b in B])
        Cm = (Mat * len(C))(*[c.mat for c in C])
        evp = None
        if stage_events is not None:
            evp = (ctypes.c_void_p * STAGE_EVENTS)(*[int(e.cuda_event) for e in stage_events])
        ws_ptr, ws_n = (workspace if isinstance(workspace, tuple)
                        else (_tensor_ptr(workspace), workspace.numel()))
        _call("pcmm_plan_run_selected", self.h, w, len(which), Bm, Cm, ws_ptr, ws_n, evp, stream_ptr(stream))


class DlogTable:
    """Baby-step table for pcmm_decrypt (j G, j < 2^log2_baby, hash index on x)."""

    def __init__(self, log2_baby: int = 20, stream=None):
        import torch
        self.log2 = log2_baby
        n = ctypes.c_size_t()
        _call("pcmm_dlog_table_bytes", log2_baby, ctypes.byref(n))
        self.t = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        w = ctypes.c_size_t()
        _call("pcmm_dlog_table_workspace", log2_baby, ctypes.byref(w))
        ws = _workspace(w.value)
        _call("pcmm_dlog_table_build", log2_baby, _tensor_ptr(self.t), self.t.numel(), _tensor_ptr(ws), ws.numel(),
              stream_ptr(stream))
        self._keep = ws


def decrypt(sk: bytes, C: DevPoints, bound: int, table: DlogTable, stream=None, workspace=None):
    """Integers m with C = Enc(m), |m| <= bound (int64 device tensor, rows x
    cols; INT64_MIN where no such m)."""
    import torch
    assert C.form == AFFINE and C.npts == 2
    out = torch.empty((C.rows, C.cols), dtype=torch.int64, device="cuda")
    n = ctypes.c_size_t()
    _call("pcmm_decrypt_workspace", C.rows * C.cols, bound, table.log2, ctypes.byref(n))
    ws = workspace if workspace is not None else _workspace(n.value)
    _call("pcmm_decrypt", sk, C.ref(), bound, _tensor_ptr(table.t), table.t.numel(), table.log2,
          _tensor_ptr(out), _tensor_ptr(ws), ws.numel(), stream_ptr(stream))
    return out
