"""Python binding of the C ABI declared in include/pvfl.h.

Argument marshalling only: torch tensors provide device memory (their
data_ptr()) and the current HIP stream; every step of the computation runs in
the HIP library libpvfl.so.  Importing works without a GPU; any call that
needs the library raises if libpvfl.so has not been built.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpvfl.so")

PLAN_HYBRID, PLAN_DIAG, PLAN_ROW, PLAN_CTMAT, PLAN_COL = 0, 1, 2, 3, 4
TIMING_DIAG, TIMING_ENCODE, TIMING_MODUP, TIMING_MODDOWN = 0, 1, 2, 3

_STATUS = {0: "OK", -1: "PVFL_E_INVALID", -2: "PVFL_E_SHAPE", -3: "PVFL_E_LEVEL", -4: "PVFL_E_NOKEY",
           -5: "PVFL_E_NOMEM", -6: "PVFL_E_DEVICE", -7: "PVFL_E_PLAN"}


class PvflError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("n_q", ctypes.c_uint32), ("n_p", ctypes.c_uint32),
                ("q", ctypes.POINTER(ctypes.c_uint64)), ("p", ctypes.POINTER(ctypes.c_uint64)),
                ("log2_scale", ctypes.c_double)]


PLAN_FEATURES = 27
OPERAND_CT_VEC, OPERAND_CT_MAT = 0, 1
OUT_ROWS, OUT_SLOTS = 0, 1
COST_TERMS = 8
COST_NAMES = ("mult", "add", "rot", "hstrot", "modup", "moddown", "pt_limbs", "const")


class PlanOpts(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("m", ctypes.c_int32), ("n", ctypes.c_int32), ("n_out", ctypes.c_int32),
                ("level", ctypes.c_int32), ("lazy_moddown", ctypes.c_int32), ("ras_in_ct", ctypes.c_int32),
                ("pack", ctypes.c_int32), ("pt_log2_scale", ctypes.c_double), ("bsgs", ctypes.c_int32),
                ("unhoisted", ctypes.c_int32)]


class Candidate(ctypes.Structure):
    _fields_ = [("opts", PlanOpts), ("batch", ctypes.c_int32)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("group", ctypes.c_int32), ("chunk", ctypes.c_int32), ("vec", ctypes.c_int32),
                ("chunk_major", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("kind", "m", "n", "n_out", "m_pad", "n_pad", "mprime", "groups",
                                              "row_blocks", "col_blocks", "n_pts", "pt_limbs", "ct_in", "ct_out",
                                              "in_level", "out_level", "n_galois")] + \
               [(n, ctypes.c_int64) for n in ("n_add", "n_mult", "n_rot", "n_hstrot")] + \
               [("out_log2_scale", ctypes.c_double)] + \
               [(n, ctypes.c_int32) for n in ("bsgs", "n_modup", "n_moddown")]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None
_VP = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        # torch bundles its own HIP runtime with the same soname as the system
        # one; loading torch first makes libpvfl bind to that single runtime,
        # so torch tensors and library calls share one device context.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        L.pvfl_last_error.restype = ctypes.c_char_p
        i32, u64, u32, sz = ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_size_t
        sig = {
            "pvfl_context_create": [ctypes.POINTER(Params), ctypes.c_int, ctypes.POINTER(_VP)],
            "pvfl_keygen": [_VP, u64, ctypes.POINTER(_VP)],
            "pvfl_rotkeys_gen": [_VP, _VP, ctypes.POINTER(u32), i32, u64, _VP, sz, ctypes.POINTER(_VP)],
            "pvfl_plan_create": [_VP, ctypes.POINTER(PlanOpts), ctypes.POINTER(_VP)],
            "pvfl_plan_get_info": [_VP, ctypes.POINTER(PlanInfo)],
            "pvfl_plan_galois": [_VP, ctypes.POINTER(u32), i32],
            "pvfl_matmul_ct_pt": [_VP, _VP, _VP, _VP, _VP, _VP, sz, _VP],
            "pvfl_matmul_ct_pt_noalloc": [_VP, _VP, _VP, _VP, _VP, _VP],
            "pvfl_pt_import": [_VP, i32, i32, _VP, i32, _VP, _VP],
            "pvfl_encrypt_coeffs": [_VP, _VP, i32, _VP, u64, _VP, _VP],
            "pvfl_export_coeffs": [_VP, i32, i32, _VP, i32, _VP, _VP],
            "pvfl_decrypt_coeffs": [_VP, _VP, i32, _VP, _VP, _VP],
            "pvfl_sk_export": [_VP, _VP, _VP],
            "pvfl_rotkeys_export": [_VP, i32, _VP, _VP],
            "pvfl_rotate": [_VP, _VP, i32, _VP, u32, i32, _VP, _VP],
            "pvfl_rescale": [_VP, i32, _VP, _VP, _VP],
            "pvfl_ct_mul_pt": [_VP, i32, _VP, _VP, _VP, _VP],
            "pvfl_ct_add": [_VP, i32, _VP, _VP, _VP, _VP],
            "pvfl_encode_pt": [_VP, _VP, ctypes.c_int64, _VP, _VP],
            "pvfl_encode_pt_scaled": [_VP, _VP, ctypes.c_int64, ctypes.c_double, _VP, _VP],
            "pvfl_pk_gen": [_VP, _VP, u64, ctypes.POINTER(_VP)],
            "pvfl_pk_export": [_VP, _VP, _VP],
            "pvfl_encrypt_pk": [_VP, _VP, _VP, ctypes.c_int64, u64, _VP, _VP],
            "pvfl_encrypt_coeffs_pk": [_VP, _VP, i32, _VP, u64, _VP, _VP],
            "pvfl_matmul_ct_pt_sum": [_VP, i32, ctypes.POINTER(_VP), ctypes.POINTER(_VP), _VP, _VP, _VP, sz, _VP],
            "pvfl_encode_out": [_VP, _VP, i32, _VP, _VP],
            "pvfl_out_add_pt": [_VP, _VP, _VP, i32, _VP, _VP],
            "pvfl_lazy_ras": [_VP, _VP, _VP, _VP],
            "pvfl_encrypt": [_VP, _VP, _VP, ctypes.c_int64, u64, _VP, _VP],
            "pvfl_decrypt_decode": [_VP, _VP, _VP, _VP, _VP],
            "pvfl_timing_enable": [_VP, i32],
            "pvfl_mlp_create": [i32, i32, i32, u64, ctypes.POINTER(_VP)],
            "pvfl_ctmat_transpose_galois": [_VP, ctypes.POINTER(u32), i32, ctypes.POINTER(i32)],
            "pvfl_ctmat_transpose": [_VP, _VP, _VP, _VP, _VP],
            "pvfl_plan_candidates": [_VP, i32, i32, i32, i32, i32, ctypes.POINTER(Candidate), i32, ctypes.POINTER(i32)],
            "pvfl_plan_features": [_VP, i32, ctypes.POINTER(ctypes.c_float), i32],
            "pvfl_plan_analytic_ms": [_VP, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
            "pvfl_planner_create": [_VP, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                    ctypes.c_float, ctypes.c_float, ctypes.POINTER(_VP)],
            "pvfl_plan_choose": [_VP, _VP, i32, i32, i32, i32, i32, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(Candidate), ctypes.POINTER(ctypes.c_double), _VP],
            "pvfl_mlp_get_params": [_VP, _VP, _VP],
            "pvfl_mlp_set_params": [_VP, _VP, _VP],
            "pvfl_mlp_forward": [_VP, _VP, i32, _VP, _VP],
            "pvfl_mlp_grad": [_VP, _VP, _VP, i32, _VP, _VP, _VP],
            "pvfl_mlp_train_step": [_VP, _VP, _VP, i32, ctypes.c_float, _VP, _VP],
            "pvfl_batch_create": [_VP, i32, ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                                  ctypes.POINTER(_VP), _VP, ctypes.POINTER(BatchOpts), _VP, sz, ctypes.POINTER(_VP)],
            "pvfl_batch_workspace_bytes": [_VP, i32, ctypes.POINTER(_VP), ctypes.POINTER(BatchOpts),
                                           ctypes.POINTER(sz)],
            "pvfl_batch_encode": [_VP, _VP],
            "pvfl_batch_encrypt": [_VP, _VP, u64, _VP],
            "pvfl_batch_matmul": [_VP, _VP],
            "pvfl_batch_decrypt": [_VP, _VP, _VP],
            "pvfl_batch_run": [_VP, _VP, u64, i32, _VP],
            "pvfl_batch_info": [_VP, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double)],
            "pvfl_timing_read": [_VP, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(ctypes.c_double)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        for name in ("pvfl_bytes_ct_in", "pvfl_bytes_ct_out", "pvfl_bytes_pt", "pvfl_bytes_workspace",
                     "pvfl_bytes_pt_out"):
            f = getattr(L, name)
            f.argtypes = [_VP]
            f.restype = sz
        L.pvfl_noalloc_max_bytes.argtypes = []
        L.pvfl_noalloc_max_bytes.restype = sz
        L.pvfl_bytes_rotkeys.argtypes = [_VP, i32]
        L.pvfl_bytes_rotkeys.restype = sz
        L.pvfl_bytes_workspace_sum.argtypes = [_VP, i32]
        L.pvfl_bytes_workspace_sum.restype = sz
        L.pvfl_mlp_num_params.argtypes = [_VP]
        L.pvfl_mlp_num_params.restype = i32
        L.pvfl_plan_num_features.argtypes = []
        L.pvfl_plan_num_features.restype = i32
        for name in ("pvfl_context_destroy", "pvfl_sk_destroy", "pvfl_pk_destroy", "pvfl_rotkeys_destroy",
                     "pvfl_plan_destroy",
                     "pvfl_batch_destroy", "pvfl_mlp_destroy", "pvfl_planner_destroy"):
            f = getattr(L, name)
            f.argtypes = [_VP]
            f.restype = None
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise PvflError(status, lib().pvfl_last_error().decode())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


E_INVALID, E_SHAPE = -1, -2


def _dev(t, what: str, nbytes: int = 0, dtype: str = "float64") -> ctypes.c_void_p:
    """the device pointer of t after checking that it is a contiguous device
    tensor of the given dtype holding at least nbytes; the library reads and
    writes raw device memory, so a wrong tensor is refused here instead"""
    if t is None:
        raise PvflError(E_INVALID, f"{what}: a device tensor is required")
    if str(t.dtype) != "torch." + dtype or not t.is_cuda or not t.is_contiguous():
        raise PvflError(E_INVALID, f"{what}: expected a contiguous {dtype} device tensor, got {t.dtype} "
                                   f"on {t.device}{'' if t.is_contiguous() else ', not contiguous'}")
    have = t.numel() * t.element_size()
    if have < nbytes:
        raise PvflError(E_SHAPE, f"{what}: {have} bytes, the call needs {nbytes}")
    return ctypes.c_void_p(t.data_ptr())


def _dev_rows(t, what: str, rows: int, cols: int):
    """a float64 device matrix of at least rows x cols with unit column stride
    (a vector counts as one row); returns (pointer, row stride)"""
    if t is None or str(t.dtype) != "torch.float64" or not t.is_cuda:
        raise PvflError(E_INVALID, f"{what}: expected a float64 device tensor")
    if t.dim() == 1:
        if rows > 1 or t.numel() < cols or t.stride(0) != 1:
            raise PvflError(E_SHAPE, f"{what}: a vector of {t.numel()} cannot hold {rows} x {cols}")
        return ctypes.c_void_p(t.data_ptr()), t.numel()
    if t.dim() != 2 or t.stride(1) != 1 or t.shape[0] < rows or t.shape[1] < cols or t.stride(0) < t.shape[1]:
        raise PvflError(E_SHAPE, f"{what}: need a row-major {rows} x {cols} matrix with unit column stride, "
                                 f"got shape {tuple(t.shape)} strides {tuple(t.stride())}")
    return ctypes.c_void_p(t.data_ptr()), t.stride(0)


class _Handle:
    _destroy = ""

    def __init__(self, h, keep=()):
        self.h = h
        self._keep = keep

    def close(self):
        if self.h is not None and self.h.value:
            getattr(lib(), self._destroy)(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context(_Handle):
    _destroy = "pvfl_context_destroy"

    def __init__(self, logN: int, q, p, log2_scale: float, device: int = 0):
        self.logN, self.N = logN, 1 << logN
        self.device = device
        self.q, self.p = [int(x) for x in q], [int(x) for x in p]
        self.log2_scale = log2_scale
        qa = (ctypes.c_uint64 * len(self.q))(*self.q)
        pa = (ctypes.c_uint64 * len(self.p))(*self.p)
        prm = Params(logN, len(self.q), len(self.p), qa, pa, log2_scale)
        h = _VP()
        _check(lib().pvfl_context_create(ctypes.byref(prm), device, ctypes.byref(h)))
        super().__init__(h)

    @staticmethod
    def from_dict(d: dict, device: int = 0) -> "Context":
        return Context(int(d["logN"]), d["q"], d["p"], float(d["log2_scale"]), device)

    @property
    def L(self) -> int:
        return len(self.q) - 1

    @property
    def alpha(self) -> int:
        return len(self.p)

    def keygen(self, seed: int) -> "SecretKey":
        h = _VP()
        _check(lib().pvfl_keygen(self.h, seed, ctypes.byref(h)))
        return SecretKey(h, keep=(self,))

    def pk_gen(self, sk: "SecretKey", seed: int) -> "PublicKey":
        h = _VP()
        _check(lib().pvfl_pk_gen(self.h, sk.h, seed, ctypes.byref(h)))
        return PublicKey(h, keep=(self,))

    def rotkeys(self, sk: "SecretKey", galois, seed: int) -> "RotKeys":
        """rotation keys for the Galois elements, in a torch device buffer this
        handle keeps alive"""
        import torch
        g = [int(x) for x in galois]
        arr = (ctypes.c_uint32 * max(1, len(g)))(*g)
        nb = int(lib().pvfl_bytes_rotkeys(self.h, len(set(g))))
        buf = torch.empty(nb, dtype=torch.uint8, device=f"cuda:{self.device}")
        h = _VP()
        _check(lib().pvfl_rotkeys_gen(self.h, sk.h, arr, len(g), seed, ctypes.c_void_p(buf.data_ptr()), nb,
                                      ctypes.byref(h)))
        return RotKeys(h, list(dict.fromkeys(g)), keep=(self, buf))

    def candidates(self, m: int, n: int, level: int = -1, operand: int = 0, n_out: int = 0) -> list:
        """every valid candidate: option dict plus "batch" (products it runs)"""
        cap = 64
        arr = (Candidate * cap)()
        cnt = ctypes.c_int32()
        _check(lib().pvfl_plan_candidates(self.h, operand, m, n, n_out, level, arr, cap, ctypes.byref(cnt)))
        return [cand_dict(arr[i]) for i in range(cnt.value)]

    def plan_from(self, o: dict) -> "Plan":
        return self.plan(o["kind"], o["m"], o["n"], n_out=o.get("n_out", 0), level=o.get("level", -1),
                         lazy=bool(o.get("lazy_moddown", 1)), ras_in_ct=bool(o.get("ras_in_ct", 0)),
                         pack=o.get("pack", 1), pt_log2_scale=o.get("pt_log2_scale", 0.0), bsgs=o.get("bsgs", 0),
                         unhoisted=bool(o.get("unhoisted", 0)))

    def plan(self, kind: int, m: int, n: int, n_out: int = 0, level: int = -1, lazy: bool = True,
             ras_in_ct: bool = False, pack: int = 1, pt_log2_scale: float = 0.0, bsgs: int = 0,
             unhoisted: bool = False) -> "Plan":
        o = PlanOpts(kind, m, n, n_out, level, int(lazy), int(ras_in_ct), pack, pt_log2_scale, bsgs, int(unhoisted))
        h = _VP()
        _check(lib().pvfl_plan_create(self.h, ctypes.byref(o), ctypes.byref(h)))
        return Plan(h, self)

    def timing_enable(self, on: bool):
        _check(lib().pvfl_timing_enable(self.h, int(on)))

    def timing_read(self, cls: int):
        """(total_ms, launches, algorithmic_bytes) of one kernel class; clears it"""
        ms, n, by = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        _check(lib().pvfl_timing_read(self.h, cls, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by)))
        return ms.value, n.value, by.value

    # byte sizes of residue arrays at a level
    def _limbs(self, level: int, with_p: bool = False) -> int:
        lv = self.L if level < 0 else level
        return lv + 1 + (self.alpha if with_p else 0)

    def _ct_bytes(self, level: int) -> int:
        return 16 * self._limbs(level) * self.N

    # integer-level entries
    def pt_import(self, level: int, with_p: bool, m_i64, out):
        count = m_i64.shape[0]
        m = _dev(m_i64, "coefficients", 8 * count * self.N, "int64")
        o = _dev(out, "plaintexts", 8 * count * self._limbs(level, with_p) * self.N)
        _check(lib().pvfl_pt_import(self.h, level, int(with_p), m, count, o, _stream()))

    def encrypt_coeffs(self, sk, level: int, m_i64, seed: int, out):
        m = _dev(m_i64, "coefficients", 8 * self.N, "int64")
        o = _dev(out, "ciphertext", self._ct_bytes(level))
        _check(lib().pvfl_encrypt_coeffs(self.h, sk.h, level, m, seed, o, _stream()))

    def encrypt_coeffs_pk(self, pk, level: int, m_i64, seed: int, out):
        m = _dev(m_i64, "coefficients", 8 * self.N, "int64")
        o = _dev(out, "ciphertext", self._ct_bytes(level))
        _check(lib().pvfl_encrypt_coeffs_pk(self.h, pk.h, level, m, seed, o, _stream()))

    def export_coeffs(self, level: int, with_p: bool, poly, count: int, out):
        nb = 8 * count * self._limbs(level, with_p) * self.N
        src = _dev(poly, "polynomials", nb)
        o = _dev(out, "residues", nb, "int64")
        _check(lib().pvfl_export_coeffs(self.h, level, int(with_p), src, count, o, _stream()))

    def decrypt_coeffs(self, sk, level: int, ct, out):
        c = _dev(ct, "ciphertext", self._ct_bytes(level))
        o = _dev(out, "residues", 8 * self._limbs(level) * self.N, "int64")
        _check(lib().pvfl_decrypt_coeffs(self.h, sk.h, level, c, o, _stream()))

    def rotate(self, keys, level: int, ct, galois: int, hoisted: bool, out):
        nb = self._ct_bytes(level)
        c, o = _dev(ct, "ciphertext", nb), _dev(out, "output", nb)
        _check(lib().pvfl_rotate(self.h, keys.h, level, c, galois, int(hoisted), o, _stream()))

    def rescale(self, level: int, ct, out):
        c = _dev(ct, "ciphertext", self._ct_bytes(level))
        o = _dev(out, "output", self._ct_bytes(level - 1) if level >= 1 else 0)
        _check(lib().pvfl_rescale(self.h, level, c, o, _stream()))

    def ct_mul_pt(self, level: int, ct, pt, out):
        nb = self._ct_bytes(level)
        c, o = _dev(ct, "ciphertext", nb), _dev(out, "output", nb)
        q = _dev(pt, "plaintext", nb // 2)
        _check(lib().pvfl_ct_mul_pt(self.h, level, c, q, o, _stream()))

    def ct_add(self, level: int, a, b, out):
        nb = self._ct_bytes(level)
        _check(lib().pvfl_ct_add(self.h, level, _dev(a, "a", nb), _dev(b, "b", nb), _dev(out, "output", nb),
                                 _stream()))


class SecretKey(_Handle):
    _destroy = "pvfl_sk_destroy"

    def export(self, out):
        ctx = self._keep[0]
        _check(lib().pvfl_sk_export(self.h, _dev(out, "residues", 8 * ctx._limbs(-1, True) * ctx.N, "int64"),
                                    _stream()))


class PublicKey(_Handle):
    _destroy = "pvfl_pk_destroy"

    def export(self, out):
        ctx = self._keep[0]
        _check(lib().pvfl_pk_export(self.h, _dev(out, "residues", ctx._ct_bytes(-1), "int64"), _stream()))


class RotKeys(_Handle):
    _destroy = "pvfl_rotkeys_destroy"

    def __init__(self, h, galois, keep=()):
        super().__init__(h, keep)
        self.galois = galois

    def export(self, index: int, out):
        ctx = self._keep[0]
        beta = -(-(ctx.L + 1) // ctx.alpha)
        nb = 8 * beta * 2 * ctx._limbs(-1, True) * ctx.N
        _check(lib().pvfl_rotkeys_export(self.h, index, _dev(out, "residues", nb, "int64"), _stream()))


class Plan(_Handle):
    _destroy = "pvfl_plan_destroy"

    def __init__(self, h, ctx: Context):
        super().__init__(h, keep=(ctx,))
        self.ctx = ctx
        info = PlanInfo()
        _check(lib().pvfl_plan_get_info(self.h, ctypes.byref(info)))
        self.info = info.as_dict()

    def galois(self) -> list:
        n = self.info["n_galois"]
        arr = (ctypes.c_uint32 * max(1, n))()
        _check(lib().pvfl_plan_galois(self.h, arr, n))
        return [int(arr[i]) for i in range(n)]

    def bytes(self, what: str) -> int:
        return int(getattr(lib(), "pvfl_bytes_" + what)(self.h))

    def _n_results(self) -> int:
        i = self.info
        return i["m"] * i["n_out"] if i["kind"] == PLAN_CTMAT else i["m"]

    def _matrix(self, X, what: str):
        """the plaintext matrix (W, n x n_out, for CTMAT): pointer and row stride"""
        i = self.info
        rows, cols = (i["n"], i["n_out"]) if i["kind"] == PLAN_CTMAT else (i["m"], i["n"])
        return _dev_rows(X, what, rows, cols)

    def _vector(self, v, what: str):
        """the encrypted operand (A, m x n, for CTMAT; else y of length n): pointer and row stride"""
        i = self.info
        if i["kind"] == PLAN_CTMAT:
            return _dev_rows(v, what, i["m"], i["n"])
        return _dev_rows(v.reshape(-1) if v is not None and v.dim() == 1 else v, what, 1, i["n"])

    def encode_pt(self, X, out, coef: float = 1.0):
        """X: device float64 matrix (row-major, unit column stride); coef scales it (Eq. 4's q_1 X)."""
        x, ld = self._matrix(X, "plaintext matrix")
        o = _dev(out, "plaintexts", self.bytes("pt"))
        if coef == 1.0:
            _check(lib().pvfl_encode_pt(self.h, x, ld, o, _stream()))
        else:
            _check(lib().pvfl_encode_pt_scaled(self.h, x, ld, float(coef), o, _stream()))

    def matmul_sum(self, cts, pts, keys, out, ws=None):
        """Eq. 4: out = sum_k product(cts[k], pts[k]) with one ModDown per output"""
        n = len(cts)
        if len(pts) != n:
            raise PvflError(E_INVALID, "one plaintext set per ciphertext set")
        ca = (_VP * n)(*[_dev(t, f"ciphertexts {k}", self.bytes("ct_in")).value for k, t in enumerate(cts)])
        pa = (_VP * n)(*[_dev(t, f"plaintexts {k}", self.bytes("pt")).value for k, t in enumerate(pts)])
        o = _dev(out, "output", self.bytes("ct_out"))
        if ws is None:
            ws = self.workspace(n)
        w = _dev(ws, "workspace", self.workspace_sum_bytes(n), str(ws.dtype)[6:]) if ws is not None else _ptr(None)
        ws_bytes = 0 if ws is None else ws.numel() * ws.element_size()
        _check(lib().pvfl_matmul_ct_pt_sum(self.h, n, ca, pa, keys.h if keys is not None else None, o, w, ws_bytes,
                                           _stream()))

    def workspace_sum_bytes(self, count: int) -> int:
        return int(lib().pvfl_bytes_workspace_sum(self.h, count))

    def _slots_bytes(self) -> int:
        return 8 * self.info["ct_out"] * (self.ctx.N // 2)

    def encode_out(self, v, mode: int, out):
        """cleartext at the output scale: mode OUT_ROWS (m values, inverse RaS) or OUT_SLOTS ([ct_out][N/2])"""
        nb = self._slots_bytes() if mode == OUT_SLOTS else 8 * self._n_results()
        _check(lib().pvfl_encode_out(self.h, _dev(v, "values", nb), mode, _dev(out, "plaintext", self.bytes("pt_out")),
                                     _stream()))

    def out_add_pt(self, ct, pt, sign: int, out):
        nb = self.bytes("ct_out")
        _check(lib().pvfl_out_add_pt(self.h, _dev(ct, "ciphertexts", nb), _dev(pt, "plaintext", self.bytes("pt_out")),
                                     sign, _dev(out, "output", nb), _stream()))

    def lazy_ras(self, slots, out):
        """the masking party's share: lazy rotate-and-sum of cleartext slots [ct_out][N/2]"""
        _check(lib().pvfl_lazy_ras(self.h, _dev(slots, "slots", self._slots_bytes()),
                                   _dev(out, "results", 8 * self._n_results()), _stream()))

    def encrypt(self, sk, v, seed: int, out):
        x, ld = self._vector(v, "encrypted operand")
        _check(lib().pvfl_encrypt(self.h, sk.h, x, ld, seed, _dev(out, "ciphertexts", self.bytes("ct_in")), _stream()))

    def encrypt_pk(self, pk, v, seed: int, out):
        x, ld = self._vector(v, "encrypted operand")
        _check(lib().pvfl_encrypt_pk(self.h, pk.h, x, ld, seed, _dev(out, "ciphertexts", self.bytes("ct_in")),
                                     _stream()))

    def decrypt_decode(self, sk, ct, out):
        _check(lib().pvfl_decrypt_decode(self.h, sk.h, _dev(ct, "ciphertexts", self.bytes("ct_out")),
                                         _dev(out, "results", 8 * self._n_results()), _stream()))

    def transpose_galois(self) -> list:
        """Galois elements the transposed diagonal conversion (Eq. 7) needs"""
        cap = 8192
        arr = (ctypes.c_uint32 * cap)()
        cnt = ctypes.c_int32()
        _check(lib().pvfl_ctmat_transpose_galois(self.h, arr, cap, ctypes.byref(cnt)))
        return [int(arr[i]) for i in range(cnt.value)]

    def transpose(self, ct_in, keys, ct_out):
        """[[A]] diagonals -> [[A^T]] diagonals (Eq. 7)"""
        nb = self.bytes("ct_in")
        _check(lib().pvfl_ctmat_transpose(self.h, _dev(ct_in, "ciphertexts", nb), keys.h if keys is not None else None,
                                          _dev(ct_out, "output", nb), _stream()))

    def features(self, batch: int = 1) -> list:
        arr = (ctypes.c_float * PLAN_FEATURES)()
        _check(lib().pvfl_plan_features(self.h, batch, arr, PLAN_FEATURES))
        return [float(x) for x in arr]

    def analytic_ms(self, costs, batch: int = 1) -> float:
        c = (ctypes.c_double * COST_TERMS)(*costs)
        out = ctypes.c_double()
        _check(lib().pvfl_plan_analytic_ms(self.h, batch, c, ctypes.byref(out)))
        return out.value

    def workspace(self, count: int = 1):
        """a device workspace for this plan's products (count terms), kept with
        the plan and reused; None for plans that need none"""
        import torch
        nb = self.bytes("workspace") if count == 1 else self.workspace_sum_bytes(count)
        if self.info["kind"] in (PLAN_CTMAT, PLAN_COL):
            return None
        if getattr(self, "_ws", None) is None or self._ws.numel() < nb:
            self._ws = torch.empty(nb, dtype=torch.uint8, device=f"cuda:{self.ctx.device}")
        return self._ws

    def matmul(self, ct, pt, keys, out, ws=None):
        c = _dev(ct, "ciphertexts", self.bytes("ct_in"))
        p = _dev(pt, "plaintexts", self.bytes("pt"))
        o = _dev(out, "output", self.bytes("ct_out"))
        if ws is None:
            ws = self.workspace()
        w = _dev(ws, "workspace", self.bytes("workspace"), str(ws.dtype)[6:]) if ws is not None else _ptr(None)
        ws_bytes = 0 if ws is None else ws.numel() * ws.element_size()
        _check(lib().pvfl_matmul_ct_pt(self.h, c, p, keys.h if keys is not None else None, o, w, ws_bytes, _stream()))

    def matmul_noalloc(self, ct, pt, keys, out):
        """pvfl_matmul_ct_pt with its workspace in the library's fixed device
        array: nothing is allocated during the call"""
        c = _dev(ct, "ciphertexts", self.bytes("ct_in"))
        p = _dev(pt, "plaintexts", self.bytes("pt"))
        o = _dev(out, "output", self.bytes("ct_out"))
        _check(lib().pvfl_matmul_ct_pt_noalloc(self.h, c, p, keys.h if keys is not None else None, o, _stream()))


def noalloc_max_bytes() -> int:
    """size of the fixed scratch array the allocation-free product uses"""
    return int(lib().pvfl_noalloc_max_bytes())


def choose_analytic(ctx: Context, m: int, n: int, costs, level: int = -1, operand: int = 0, n_out: int = 0):
    """the candidate of least analytic latency (no network needed)"""
    c = (ctypes.c_double * COST_TERMS)(*costs)
    k = Candidate()
    pred = ctypes.c_double()
    _check(lib().pvfl_plan_choose(None, ctx.h, operand, m, n, n_out, level, c, ctypes.byref(k), ctypes.byref(pred),
                                  _stream()))
    return cand_dict(k), pred.value


def opts_dict(o: PlanOpts) -> dict:
    return {name: getattr(o, name) for name, _ in o._fields_}


def cand_dict(k: Candidate) -> dict:
    d = opts_dict(k.opts)
    d["batch"] = int(k.batch)
    return d


class Planner(_Handle):
    """Native plan selection: the latency network (or, with costs, the
    analytic operation-count model) ranks every candidate plan."""
    _destroy = "pvfl_planner_destroy"

    def __init__(self, mlp: "Mlp", x_mean, x_std, y_mean: float, y_std: float):
        xm = (ctypes.c_float * PLAN_FEATURES)(*x_mean)
        xs = (ctypes.c_float * PLAN_FEATURES)(*x_std)
        h = _VP()
        _check(lib().pvfl_planner_create(mlp.h if mlp is not None else None, xm, xs, y_mean, y_std, ctypes.byref(h)))
        super().__init__(h, keep=(mlp,))

    def choose(self, ctx: Context, m: int, n: int, level: int = -1, costs=None, operand: int = 0, n_out: int = 0):
        c = (ctypes.c_double * COST_TERMS)(*costs) if costs is not None else None
        k = Candidate()
        pred = ctypes.c_double()
        _check(lib().pvfl_plan_choose(self.h, ctx.h, operand, m, n, n_out, level, c, ctypes.byref(k),
                                      ctypes.byref(pred), _stream()))
        return cand_dict(k), pred.value


def _ptr_array(items):
    arr = (_VP * len(items))()
    for i, t in enumerate(items):
        arr[i] = t.data_ptr() if t is not None else None
    return arr


class Batch(_Handle):
    """Many independent products run phase by phase in single launches."""
    _destroy = "pvfl_batch_destroy"

    def __init__(self, ctx: Context, plans, X=None, v=None, pt=None, ct=None, out=None, y=None, keys=None,
                 group: int = 2, chunk: int = 32, vec: int = 1, chunk_major: bool = True, ws=None):
        import torch
        n = len(plans)
        plan_arr = (_VP * n)(*[p.h.value for p in plans])
        opts = BatchOpts(group, chunk, vec, int(chunk_major))
        need = ctypes.c_size_t()
        _check(lib().pvfl_batch_workspace_bytes(ctx.h, n, plan_arr, ctypes.byref(opts), ctypes.byref(need)))
        if ws is None:
            ws = torch.empty(need.value, dtype=torch.uint8, device=f"cuda:{ctx.device}")
        wsp = _dev(ws, "workspace", need.value, str(ws.dtype)[6:])
        for name, lst in (("pt", pt), ("ct", ct), ("out", out), ("X", X), ("v", v), ("y", y)):
            if lst is not None and len(lst) != n:
                raise PvflError(E_INVALID, f"{name}: one entry per product")
        ld = (ctypes.c_int64 * n)()
        for k, p in enumerate(plans):
            _dev(pt[k], f"plaintexts {k}", p.bytes("pt"))
            _dev(ct[k], f"ciphertext {k}", p.bytes("ct_in"))
            _dev(out[k], f"output {k}", p.bytes("ct_out"))
            if X is not None:
                ld[k] = p._matrix(X[k], f"plaintext matrix {k}")[1]
            if v is not None:
                p._vector(v[k], f"encrypted vector {k}")
            if y is not None:
                _dev(y[k], f"results {k}", 8 * p._n_results())
        h = _VP()
        _check(lib().pvfl_batch_create(ctx.h, n, plan_arr,
                                       _ptr_array(X) if X is not None else None, ld,
                                       _ptr_array(v) if v is not None else None,
                                       _ptr_array(pt), _ptr_array(ct), _ptr_array(out),
                                       _ptr_array(y) if y is not None else None,
                                       keys.h if keys is not None else None,
                                       ctypes.byref(opts), wsp, ws.numel() * ws.element_size(), ctypes.byref(h)))
        super().__init__(h, keep=(ctx, plans, X, v, pt, ct, out, y, keys, ws))
        self.workspace_bytes = need.value

    def encode(self):
        _check(lib().pvfl_batch_encode(self.h, _stream()))

    def encrypt(self, sk, seed: int):
        _check(lib().pvfl_batch_encrypt(self.h, sk.h, seed, _stream()))

    def matmul(self):
        _check(lib().pvfl_batch_matmul(self.h, _stream()))

    def decrypt(self, sk):
        _check(lib().pvfl_batch_decrypt(self.h, sk.h, _stream()))

    def run(self, sk, seed: int, graph: bool = False):
        _check(lib().pvfl_batch_run(self.h, sk.h, seed, int(graph), _stream()))

    def info(self):
        n, kb, pb = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        _check(lib().pvfl_batch_info(self.h, ctypes.byref(n), ctypes.byref(kb), ctypes.byref(pb)))
        return {"work_items": n.value, "key_bytes": kb.value, "pt_bytes": pb.value}


class Mlp(_Handle):
    """The plan selector's latency network (FP32, GPU-trained)."""
    _destroy = "pvfl_mlp_destroy"

    def __init__(self, n_in: int, hidden: int = 64, max_batch: int = 1024, seed: int = 0):
        h = _VP()
        _check(lib().pvfl_mlp_create(n_in, hidden, max_batch, seed, ctypes.byref(h)))
        super().__init__(h)
        self.n_in, self.hidden = n_in, hidden
        self.n_params = int(lib().pvfl_mlp_num_params(self.h))

    def get_params(self):
        import torch
        out = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(lib().pvfl_mlp_get_params(self.h, _ptr(out), _stream()))
        return out

    def set_params(self, p):
        _check(lib().pvfl_mlp_set_params(self.h, _dev(p, "parameters", 4 * self.n_params, "float32"), _stream()))

    def _check_x(self, x, t=None):
        import torch
        if x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous() or x.dim() != 2 \
                or x.shape[1] != self.n_in:
            raise ValueError(f"x must be a contiguous float32 device tensor of shape [batch, {self.n_in}]")
        if t is not None and (t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous()
                              or t.shape != (x.shape[0],)):
            raise ValueError("targets must be a contiguous float32 device vector of length batch")

    def forward(self, x):
        import torch
        self._check_x(x)
        y = torch.empty(x.shape[0], dtype=torch.float32, device="cuda")
        _check(lib().pvfl_mlp_forward(self.h, _ptr(x), x.shape[0], _ptr(y), _stream()))
        return y

    def grad(self, x, t):
        import torch
        self._check_x(x, t)
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(lib().pvfl_mlp_grad(self.h, _ptr(x), _ptr(t), x.shape[0], _ptr(g), _ptr(loss), _stream()))
        return g, loss

    def train_step(self, x, t, lr: float):
        import torch
        self._check_x(x, t)
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(lib().pvfl_mlp_train_step(self.h, _ptr(x), _ptr(t), x.shape[0], lr, _ptr(loss), _stream()))
        return loss
