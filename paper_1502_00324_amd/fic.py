"""Python binding of libfic.so (the gfx950 fractal encoder C ABI).

Argument marshalling only: every step of the encoder and decoder runs in
the library's HIP kernels.  PyTorch provides device memory and the stream.
The entry points keep the C names: build_domain_pool, encode_level, encode,
decode (see include/fic.h for the contract of each).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfic.so")

FIC_OK, FIC_E_INVALID, FIC_E_NOMEM, FIC_E_HIP, FIC_E_CAPACITY, FIC_E_ARCH, FIC_E_LIMIT = 0, -1, -2, -3, -4, -5, -6
DECODE_NOALLOC_MAX_PIXELS = 1 << 24
ENGINE_MFMA, ENGINE_FP32, ENGINE_MFMA_I8, ENGINE_MFMA_F16, ENGINE_MFMA_F16_16X16 = 0, 1, 2, 3, 4
POOL_ENTROPY, POOL_VARIANCE = 0, 1
MAX_LEVELS, MAX_S = 4, 32

i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p


class FicError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s failed: %s (%d)" % (where, strerror(status), status))


class Ratio(ctypes.Structure):
    _fields_ = [("num", i32), ("den", i32)]


class Image(ctypes.Structure):
    _fields_ = [("pix", vp), ("width", i32), ("height", i32), ("pitch", i32)]


class Params(ctypes.Structure):
    _fields_ = [("levels", i32), ("block0", i32), ("step", i32 * MAX_LEVELS), ("pool_pct", Ratio),
                ("pool_max", i32), ("s_count", i32 * MAX_LEVELS), ("s_den", i32 * MAX_LEVELS),
                ("s_num", (i32 * MAX_S) * MAX_LEVELS), ("split_rms", Ratio * MAX_LEVELS), ("engine", i32),
                ("pool_key", i32)]


T_POOL, T_PREP, T_SEARCH, T_FINAL, T_DECODE, T_KINDS = 0, 1, 2, 3, 4, 5
T_NAMES = ("pool", "prep", "search", "final", "decode")


class Timing(ctypes.Structure):
    _fields_ = [("ms", (ctypes.c_double * 6) * T_KINDS), ("launches", (i32 * 6) * T_KINDS)]


FORM_I8, FORM_F16_16X16, FORM_F16 = 0, 1, 2
FORMS = 3
FORM_NAMES = ("mfma_i8", "mfma_f16_16x16", "mfma_f16")


class Tuning(ctypes.Structure):
    _fields_ = [("choice", (i32 * 6) * FORMS)]


class PoolC(ctypes.Structure):
    _fields_ = [("capacity", i32), ("count", vp), ("xy", vp), ("key", vp), ("sum4", vp), ("a", vp)]


class CodesC(ctypes.Structure):
    _fields_ = [("capacity", i32), ("count", vp), ("xy", vp), ("split", vp), ("domain", vp), ("iso", vp),
                ("s_idx", vp), ("offset", vp), ("err", vp)]


_lib = None


def lib() -> ctypes.CDLL:
    """The HIP library; raises when it has not been built (no CPU fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libfic.so is not built (run __graft_entry__.build()); the encoder has no "
                              "other implementation")
        L = ctypes.CDLL(LIB_PATH)
        L.fic_strerror.restype = ctypes.c_char_p
        L.fic_strerror.argtypes = [i32]
        L.fic_ctx_create.argtypes = [ctypes.POINTER(vp), i32]
        L.fic_ctx_destroy.argtypes = [vp]
        L.fic_ctx_destroy.restype = None
        L.fic_ctx_set_scratch_limit.argtypes = [vp, i64]
        L.fic_ctx_set_timing.argtypes = [vp, i32]
        L.fic_ctx_set_graphs.argtypes = [vp, i32]
        L.fic_ctx_graph_count.argtypes = [vp]
        L.fic_ctx_read_timing.argtypes = [vp, ctypes.POINTER(Timing)]
        L.fic_validate_params.argtypes = [ctypes.POINTER(Params), i32, i32]
        L.fic_query_capacity.argtypes = [ctypes.POINTER(Params), i32, i32, vp, vp]
        L.fic_entropy_table.argtypes = [vp, i32]
        L.fic_level_engine.argtypes = [i32, i32]
        L.fic_pack_capacity.argtypes = [ctypes.POINTER(Params), i32, i32, vp]
        L.fic_pack.argtypes = [vp, ctypes.POINTER(Params), i32, i32, ctypes.POINTER(PoolC), ctypes.POINTER(CodesC),
                               vp, i64, vp, vp]
        L.fic_unpack_header.argtypes = [vp, i64, ctypes.POINTER(Params), vp, vp]
        L.fic_unpack.argtypes = [vp, i64, ctypes.POINTER(PoolC), ctypes.POINTER(CodesC)]
        L.fic_s_histogram.argtypes = [vp, ctypes.POINTER(Image), ctypes.POINTER(Params), ctypes.POINTER(PoolC),
                                      ctypes.POINTER(CodesC), i32, vp, vp]
        L.fic_build_domain_pool.argtypes = [vp, ctypes.POINTER(Image), i32, i32, Ratio, i32, i32, ctypes.POINTER(PoolC),
                                            vp]
        L.fic_encode_level.argtypes = [vp, ctypes.POINTER(Image), ctypes.POINTER(PoolC), vp, vp, i32, i32, vp, i32,
                                       i32, Ratio, i32, i32, ctypes.POINTER(CodesC), vp, vp, vp]
        L.fic_encode.argtypes = [vp, ctypes.POINTER(Image), i32, ctypes.POINTER(Params), ctypes.POINTER(PoolC),
                                 ctypes.POINTER(CodesC), vp]
        L.fic_decode.argtypes = [vp, ctypes.POINTER(Params), ctypes.POINTER(PoolC), ctypes.POINTER(CodesC), i32, i32,
                                 i32, vp, vp]
        L.fic_decode_noalloc.argtypes = [vp, ctypes.POINTER(Params), ctypes.POINTER(PoolC), ctypes.POINTER(CodesC),
                                         i32, i32, i32, vp, vp]
        L.fic_shape_count.argtypes = [i32, i32]
        L.fic_shape_describe.argtypes = [i32, i32, i32, vp]
        L.fic_ctx_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.fic_ctx_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.fic_autotune.argtypes = [vp, ctypes.POINTER(Image), i32, ctypes.POINTER(Params), ctypes.POINTER(PoolC),
                                   ctypes.POINTER(CodesC), i32, vp, ctypes.POINTER(Tuning)]
        _lib = L
    return _lib


EXPORTED = ("fic_ctx_create", "fic_ctx_destroy", "fic_ctx_set_scratch_limit", "fic_ctx_set_timing",
            "fic_ctx_set_graphs", "fic_ctx_graph_count",
            "fic_ctx_read_timing", "fic_strerror",
            "fic_validate_params", "fic_query_capacity", "fic_level_engine", "fic_entropy_table",
            "fic_build_domain_pool",
            "fic_encode_level", "fic_encode", "fic_decode", "fic_decode_noalloc", "fic_pack_capacity", "fic_pack", "fic_unpack_header",
            "fic_unpack", "fic_s_histogram", "fic_shape_count", "fic_shape_describe", "fic_ctx_get_tuning",
            "fic_ctx_set_tuning", "fic_autotune")


def strerror(status: int) -> str:
    return lib().fic_strerror(status).decode()


def _check(status: int, where: str):
    if status != FIC_OK:
        raise FicError(status, where)


# ---------------------------------------------------------------- parameters
def make_params(levels, block0=None, pct=(3, 10), pool_max=0, s_num=tuple(range(17)), s_den=16,
                split_rms=(8, 1), engine=ENGINE_MFMA, pool_key=POOL_ENTROPY) -> Params:
    """levels: list of (B, L).  s_num / s_den / split_rms: one value for all
    levels or one per level."""
    p = Params()
    nl = len(levels)
    p.levels = nl
    p.block0 = block0 if block0 is not None else levels[0][0]
    per_level_s = isinstance(s_num[0], (list, tuple, np.ndarray))
    for l, (B, L) in enumerate(levels):
        if B != p.block0 >> l:
            raise ValueError("level sizes must halve: %r" % (levels,))
        p.step[l] = L
        sn = s_num[l] if per_level_s else s_num
        sd = s_den[l] if isinstance(s_den, (list, tuple)) else s_den
        rm = split_rms[l] if isinstance(split_rms[0], (list, tuple)) else split_rms
        p.s_count[l] = len(sn)
        p.s_den[l] = sd
        for k, v in enumerate(sn):
            p.s_num[l][k] = int(v)
        p.split_rms[l] = Ratio(int(rm[0]), int(rm[1]))
    p.pool_pct = Ratio(int(pct[0]), int(pct[1]))
    p.pool_max = pool_max
    p.engine = engine
    p.pool_key = pool_key
    return p


def shape_count(form: int, B: int) -> int:
    """Compiled tile shapes of a matrix form at block size B (0: none)."""
    return lib().fic_shape_count(form, B)


def shape_describe(form: int, B: int, index: int) -> tuple:
    """(operand form, range quads per wave, tiles per stage, waves per SIMD)."""
    out = np.zeros(4, np.int32)
    _check(lib().fic_shape_describe(form, B, index, out.ctypes.data), "fic_shape_describe")
    return tuple(int(v) for v in out)


def tuning_dict(t: Tuning) -> dict:
    """{(form name, B): candidate} for the entries that are not -1."""
    return {(FORM_NAMES[f], 1 << l): t.choice[f][l] for f in range(FORMS) for l in range(6) if t.choice[f][l] >= 0}


def level_engine(engine: int, B: int) -> int:
    """The engine that runs a level of block size B when `engine` is asked for."""
    e = lib().fic_level_engine(engine, B)
    _check(min(e, 0), "fic_level_engine")
    return e


def validate_params(p: Params, width: int, height: int) -> int:
    return lib().fic_validate_params(ctypes.byref(p), width, height)


def query_capacity(p: Params, width: int, height: int):
    pc = np.zeros(MAX_LEVELS, np.int64)
    rc = np.zeros(MAX_LEVELS, np.int64)
    _check(lib().fic_query_capacity(ctypes.byref(p), width, height, pc.ctypes.data, rc.ctypes.data),
           "fic_query_capacity")
    return pc[:p.levels].tolist(), rc[:p.levels].tolist()


def pack_capacity(p: Params, width: int, height: int) -> int:
    out = np.zeros(1, np.int64)
    _check(lib().fic_pack_capacity(ctypes.byref(p), width, height, out.ctypes.data), "fic_pack_capacity")
    return int(out[0])


def unpack(data) -> tuple:
    """Host-side unpacking of a stream (bytes or uint8 array): (params, W, H,
    levels) with per level the pool xy and the codes as numpy arrays."""
    buf = np.frombuffer(bytes(data), np.uint8) if not isinstance(data, np.ndarray) else np.ascontiguousarray(data)
    p = Params()
    W, H = np.zeros(1, np.int32), np.zeros(1, np.int32)
    _check(lib().fic_unpack_header(buf.ctypes.data, buf.size, ctypes.byref(p), W.ctypes.data, H.ctypes.data),
           "fic_unpack_header")
    W, H = int(W[0]), int(H[0])
    pcap, rcap = query_capacity(p, W, H)
    keep, pools, codes = [], (PoolC * p.levels)(), (CodesC * p.levels)()
    for l in range(p.levels):
        arr = lambda n, dt: keep.append(np.zeros(max(n, 1), dt)) or keep[-1]
        pc, px, pk, ps, pa = arr(1, np.int32), arr(pcap[l], np.uint32), arr(pcap[l], np.int64), \
            arr(pcap[l], np.uint32), arr(pcap[l], np.int64)
        pools[l] = PoolC(pcap[l], pc.ctypes.data, px.ctypes.data, pk.ctypes.data, ps.ctypes.data, pa.ctypes.data)
        cols = [arr(1, np.int32), arr(rcap[l], np.uint32), arr(rcap[l], np.uint8), arr(rcap[l], np.uint32),
                arr(rcap[l], np.uint8), arr(rcap[l], np.uint8), arr(rcap[l], np.uint8), arr(rcap[l], np.int64)]
        codes[l] = CodesC(rcap[l], *[c.ctypes.data for c in cols])
    _check(lib().fic_unpack(buf.ctypes.data, buf.size, pools, codes), "fic_unpack")
    levels = []
    for l in range(p.levels):
        pk = keep[l * 13:(l + 1) * 13]
        dn, n = int(pk[0][0]), int(pk[5][0])
        levels.append({"pool_xy": pk[1][:dn].copy(),
                       "codes": {k: pk[6 + i][:n].copy() for i, k in
                                 enumerate(("xy", "split", "domain", "iso", "s_idx", "offset", "err"))}})
    return p, W, H, levels


def to_device(p: Params, W: int, H: int, levels: list, device):
    """Unpacked host levels -> device Pool / Codes lists for Context.decode."""
    t = _torch()
    pcap, rcap = query_capacity(p, W, H)
    pools, codes = [], []
    for l, lv in enumerate(levels):
        pl = Pool.alloc(pcap[l], device)
        n = len(lv["pool_xy"])
        pl.count.fill_(n)
        pl.xy[:n] = t.from_numpy(lv["pool_xy"].view(np.int32)).to(device)
        cd = Codes.alloc(rcap[l], device)
        c = lv["codes"]
        m = len(c["xy"])
        cd.count.fill_(m)
        for k in ("xy", "domain"):
            getattr(cd, k)[:m] = t.from_numpy(c[k].view(np.int32)).to(device)
        for k in ("split", "iso", "s_idx", "offset"):
            getattr(cd, k)[:m] = t.from_numpy(c[k]).to(device)
        cd.err[:m] = 0
        pools.append(pl)
        codes.append(cd)
    return pools, codes


def entropy_table() -> np.ndarray:
    out = np.zeros(4097, np.int64)
    _check(lib().fic_entropy_table(out.ctypes.data, 4097), "fic_entropy_table")
    return out


# ---------------------------------------------------------------- device buffers
def _torch():
    import torch
    return torch


def _stream():
    return vp(_torch().cuda.current_stream().cuda_stream)


@dataclass
class Pool:
    count: object
    xy: object
    key: object
    sum4: object
    a: object

    @staticmethod
    def alloc(cap: int, device) -> "Pool":
        t = _torch()
        return Pool(t.zeros(1, dtype=t.int32, device=device), t.empty(cap, dtype=t.int32, device=device),
                    t.empty(cap, dtype=t.int64, device=device), t.empty(cap, dtype=t.int32, device=device),
                    t.empty(cap, dtype=t.int64, device=device))

    def c(self) -> PoolC:
        return PoolC(self.xy.numel(), self.count.data_ptr(), self.xy.data_ptr(), self.key.data_ptr(),
                     self.sum4.data_ptr(), self.a.data_ptr())

    def numpy(self) -> dict:
        n = int(self.count.item())
        return {"xy": self.xy[:n].cpu().numpy().view(np.uint32), "key": self.key[:n].cpu().numpy(),
                "sum4": self.sum4[:n].cpu().numpy().view(np.uint32), "a": self.a[:n].cpu().numpy()}


@dataclass
class Codes:
    count: object
    xy: object
    split: object
    domain: object
    iso: object
    s_idx: object
    offset: object
    err: object

    @staticmethod
    def alloc(cap: int, device) -> "Codes":
        t = _torch()
        e = lambda dt: t.empty(max(cap, 1), dtype=dt, device=device)
        return Codes(t.zeros(1, dtype=t.int32, device=device), e(t.int32), e(t.uint8), e(t.int32), e(t.uint8),
                     e(t.uint8), e(t.uint8), e(t.int64))

    def c(self) -> CodesC:
        return CodesC(self.xy.numel(), self.count.data_ptr(), self.xy.data_ptr(), self.split.data_ptr(),
                      self.domain.data_ptr(), self.iso.data_ptr(), self.s_idx.data_ptr(), self.offset.data_ptr(),
                      self.err.data_ptr())

    def numpy(self) -> dict:
        n = int(self.count.item())
        return {"xy": self.xy[:n].cpu().numpy().view(np.uint32), "split": self.split[:n].cpu().numpy(),
                "domain": self.domain[:n].cpu().numpy().view(np.uint32), "iso": self.iso[:n].cpu().numpy(),
                "s_idx": self.s_idx[:n].cpu().numpy(), "offset": self.offset[:n].cpu().numpy(),
                "err": self.err[:n].cpu().numpy()}


def _image(img) -> Image:
    if img.dtype != _torch().uint8 or img.dim() != 2 or not img.is_cuda:
        raise ValueError("image must be a 2-D uint8 CUDA tensor")
    if img.stride(1) != 1:
        raise ValueError("image rows must be contiguous")
    return Image(img.data_ptr(), img.shape[1], img.shape[0], img.stride(0))


class Context:
    """Owns a fic_ctx (scratch memory) on one device."""

    def __init__(self, device: int = 0):
        self.device = device
        h = vp()
        _check(lib().fic_ctx_create(ctypes.byref(h), device), "fic_ctx_create")
        self.h = h

    def close(self):
        if self.h:
            lib().fic_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_scratch_limit(self, nbytes: int):
        _check(lib().fic_ctx_set_scratch_limit(self.h, nbytes), "fic_ctx_set_scratch_limit")

    def pack(self, p: Params, width: int, height: int, pools, codes):
        """Packs one encoded image on the device; returns (stream bytes as a
        numpy uint8 array, {header, pool, records, total} bits)."""
        t = _torch()
        dev = codes[0].xy.device
        cap = pack_capacity(p, width, height)
        out = t.empty(cap, dtype=t.uint8, device=dev)
        sizes = t.zeros(4, dtype=t.int64, device=dev)
        pc = (PoolC * p.levels)(*[pl.c() for pl in pools])
        cc = (CodesC * p.levels)(*[cd.c() for cd in codes])
        _check(lib().fic_pack(self.h, ctypes.byref(p), width, height, pc, cc, out.data_ptr(), cap,
                              sizes.data_ptr(), _stream()), "fic_pack")
        sz = sizes.cpu().tolist()
        nbytes = (sz[3] + 7) // 8
        return out[:nbytes].cpu().numpy(), dict(zip(("header_bits", "pool_bits", "record_bits", "total_bits"), sz))

    def s_histogram(self, image, p: Params, pools, codes, nbins: int = 20) -> list:
        """Per level: {'s_star': counts of the nbins bins of the chosen match's
        least-squares contrast over [0, 1), 'under', 'over', 'flat',
        's_index': counts per contrast index} over the accepted ranges."""
        t = _torch()
        per = nbins + 3 + MAX_S
        out = t.zeros(per * p.levels, dtype=t.int64, device=image.device)
        pc = (PoolC * p.levels)(*[pl.c() for pl in pools])
        cc = (CodesC * p.levels)(*[cd.c() for cd in codes])
        im = _image(image)
        _check(lib().fic_s_histogram(self.h, ctypes.byref(im), ctypes.byref(p), pc, cc, nbins, out.data_ptr(),
                                     _stream()), "fic_s_histogram")
        h = out.cpu().numpy().reshape(p.levels, per)
        return [{"under": int(r[0]), "s_star": r[1:nbins + 1].copy(), "over": int(r[nbins + 1]),
                 "flat": int(r[nbins + 2]), "s_index": r[nbins + 3:nbins + 3 + p.s_count[l]].copy()}
                for l, r in enumerate(h)]

    def set_graphs(self, max_graphs: int):
        """Capture encodes into HIP graphs and replay them for repeated arguments."""
        _check(lib().fic_ctx_set_graphs(self.h, int(max_graphs)), "fic_ctx_set_graphs")

    def graph_count(self) -> int:
        return lib().fic_ctx_graph_count(self.h)

    def get_tuning(self) -> Tuning:
        t = Tuning()
        _check(lib().fic_ctx_get_tuning(self.h, ctypes.byref(t)), "fic_ctx_get_tuning")
        return t

    def set_tuning(self, choices: dict | Tuning):
        """choices: a Tuning, or {(form name or index, B): candidate} (others: default)."""
        if isinstance(choices, Tuning):
            t = choices
        else:
            t = Tuning()
            for f in range(FORMS):
                for l in range(6):
                    t.choice[f][l] = -1
            for (form, B), c in choices.items():
                f = FORM_NAMES.index(form) if isinstance(form, str) else int(form)
                t.choice[f][int(B).bit_length() - 1] = int(c)
        _check(lib().fic_ctx_set_tuning(self.h, ctypes.byref(t)), "fic_ctx_set_tuning")

    def autotune(self, images, p: Params, bufs=None, reps: int = 3) -> dict:
        """Times every compiled tile shape of p's matrix levels on these images
        and keeps the fastest in the context.  Returns {(form, B): candidate}."""
        if bufs is None:
            bufs = self.alloc_encode([(im.shape[1], im.shape[0]) for im in images], p, images[0].device)
        n = len(images)
        imgs = (Image * n)(*[_image(im) for im in images])
        pools = (PoolC * (n * p.levels))(*[pl.c() for (pls, _) in bufs for pl in pls])
        codes = (CodesC * (n * p.levels))(*[cd.c() for (_, cds) in bufs for cd in cds])
        t = Tuning()
        _check(lib().fic_autotune(self.h, imgs, n, ctypes.byref(p), pools, codes, int(reps), _stream(),
                                  ctypes.byref(t)), "fic_autotune")
        return tuning_dict(t)

    def set_timing(self, enable: bool):
        _check(lib().fic_ctx_set_timing(self.h, int(enable)), "fic_ctx_set_timing")

    def read_timing(self) -> dict:
        """{(stage, B): (ms, launches)} summed over the recorded calls."""
        t = Timing()
        _check(lib().fic_ctx_read_timing(self.h, ctypes.byref(t)), "fic_ctx_read_timing")
        out = {}
        for k in range(T_KINDS):
            for s in range(6):
                if t.launches[k][s]:
                    out[(T_NAMES[k], 1 << s)] = (t.ms[k][s], t.launches[k][s])
        return out

    # -------------------------------------------------------------- entry points
    def build_domain_pool(self, img, B: int, L: int, pct=(3, 10), pool_max: int = 0, pool: Pool | None = None,
                          pool_key: int = POOL_ENTROPY) -> Pool:
        H, W = img.shape
        nd = ((W - 2 * B) // L + 1) * ((H - 2 * B) // L + 1)
        cap = min(nd, pool_max) if pool_max > 0 else nd
        pool = pool or Pool.alloc(cap, img.device)
        pc = pool.c()
        _check(lib().fic_build_domain_pool(self.h, ctypes.byref(_image(img)), B, L, Ratio(*pct), pool_max, pool_key,
                                           ctypes.byref(pc), _stream()), "fic_build_domain_pool")
        return pool

    def encode_level(self, img, pool: Pool, ranges_xy, n_ranges, range_cap: int, B: int, s_num, s_den: int,
                     split_rms=(8, 1), is_last: bool = False, engine: int = ENGINE_MFMA):
        """ranges_xy: int32 CUDA tensor (packed y<<16|x); n_ranges: 1-element int32
        CUDA tensor.  Returns (codes, children_xy, n_children)."""
        t = _torch()
        dev = img.device
        codes = Codes.alloc(range_cap, dev)
        children = None if is_last else t.empty(max(4 * range_cap, 1), dtype=t.int32, device=dev)
        nch = None if is_last else t.zeros(1, dtype=t.int32, device=dev)
        sn = np.ascontiguousarray(s_num, np.int32)
        cc = codes.c()
        pc = pool.c()
        _check(lib().fic_encode_level(self.h, ctypes.byref(_image(img)), ctypes.byref(pc), ranges_xy.data_ptr(),
                                      n_ranges.data_ptr(), range_cap, B, sn.ctypes.data, len(sn), s_den,
                                      Ratio(*split_rms), int(is_last), engine, ctypes.byref(cc),
                                      None if is_last else children.data_ptr(),
                                      None if is_last else nch.data_ptr(), _stream()), "fic_encode_level")
        return codes, children, nch

    def alloc_encode(self, shapes, p: Params, device):
        """Pools and codes for images of the given (width, height) shapes."""
        out = []
        for (W, H) in shapes:
            pc, rc = query_capacity(p, W, H)
            out.append(([Pool.alloc(int(c), device) for c in pc], [Codes.alloc(int(c), device) for c in rc]))
        return out

    def encode(self, images, p: Params, bufs=None):
        """images: list of 2-D uint8 CUDA tensors.  Returns, per image, the
        lists (pools, codes) of device buffers, one entry per level."""
        if bufs is None:
            bufs = self.alloc_encode([(im.shape[1], im.shape[0]) for im in images], p, images[0].device)
        n = len(images)
        imgs = (Image * n)(*[_image(im) for im in images])
        pools = (PoolC * (n * p.levels))(*[pl.c() for (pls, _) in bufs for pl in pls])
        codes = (CodesC * (n * p.levels))(*[cd.c() for (_, cds) in bufs for cd in cds])
        _check(lib().fic_encode(self.h, imgs, n, ctypes.byref(p), pools, codes, _stream()), "fic_encode")
        return bufs

    def decode(self, p: Params, pools, codes, width: int, height: int, iterations: int, out=None):
        t = _torch()
        out = out if out is not None else t.empty((height, width), dtype=t.uint8, device=codes[0].xy.device)
        pc = (PoolC * p.levels)(*[pl.c() for pl in pools])
        cc = (CodesC * p.levels)(*[cd.c() for cd in codes])
        _check(lib().fic_decode(self.h, ctypes.byref(p), pc, cc, width, height, iterations, out.data_ptr(),
                                _stream()), "fic_decode")
        return out

    def decode_noalloc(self, p: Params, pools, codes, width: int, height: int, iterations: int, out):
        """fic_decode through the allocation-free entry point: `out` must be a
        caller-allocated height x width uint8 device tensor."""
        pc = (PoolC * p.levels)(*[pl.c() for pl in pools])
        cc = (CodesC * p.levels)(*[cd.c() for cd in codes])
        _check(lib().fic_decode_noalloc(self.h, ctypes.byref(p), pc, cc, width, height, iterations,
                                        out.data_ptr(), _stream()), "fic_decode_noalloc")
        return out


def levels_numpy(pools, codes, p: Params):
    """Host copies of one image's encoder output, trimmed to the live counts."""
    out = []
    for l in range(p.levels):
        out.append({"B": p.block0 >> l, "pool": pools[l].numpy(), "codes": codes[l].numpy(),
                    "s_num": np.array(p.s_num[l][:p.s_count[l]], np.int32), "s_den": p.s_den[l]})
    return out
