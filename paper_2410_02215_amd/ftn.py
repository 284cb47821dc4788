"""Thin Python binding of libftn.so (argument marshalling only).

Every operation runs in the HIP library; this module converts Python
arguments into the C ABI declared in include/ftn.h and wraps handles. Device
buffers passed in or out are torch tensors on the current HIP device, and
work is enqueued on torch's current stream. There is no fallback: if the
library cannot be loaded, importing the operations raises.
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libftn.so")

Z2, U1, U1xU1 = 0, 1, 2
F64, F32 = 0, 1
LOCAL, GLOBAL = 0, 1
GEMM_F64, GEMM_F32, GEMM_BF16X3 = 0, 1, 2

SYM_NAMES = {"Z2": Z2, "U1": U1, "U1xU1": U1xU1}
_ERRORS = {-1: "EINVAL", -2: "ECHARGE", -3: "ENOMEM", -4: "EHIP", -5: "ENOCONV", -6: "ENOTSUP"}

_lib = None

# (name, restype, argtypes)
_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_D = ctypes.c_double
_PI32 = ctypes.POINTER(ctypes.c_int32)
_PI64 = ctypes.POINTER(ctypes.c_int64)
_PU8 = ctypes.POINTER(ctypes.c_uint8)
_PD = ctypes.POINTER(ctypes.c_double)
_PP = ctypes.POINTER(ctypes.c_void_p)

SIGNATURES = [
    ("ftn_last_error", ctypes.c_char_p, []),
    ("ftn_version", ctypes.c_char_p, []),
    ("ftn_set_allocator", _I, [_P, _P, _P]),
    ("ftn_tensor_create", _I, [_I, _I, _I, _PI32, _PI32, _PI64, _PU8, _PI32, _P, _P, _PP]),
    ("ftn_tensor_wrap", _I, [_I, _I, _I, _PI32, _PI32, _PI64, _PU8, _PI32, _P, _P, _PP]),
    ("ftn_tensor_from_dense", _I, [_I, _I, _I, _PI32, _PI32, _PI64, _PU8, _PI32, _P, _P, _PP]),
    ("ftn_tensor_to_dense", _I, [_P, _P, _P]),
    ("ftn_tensor_info", _I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I), _PI64, _PI64, _PI32]),
    ("ftn_tensor_blocks", _I, [_P, ctypes.POINTER(_PI32), ctypes.POINTER(_PI64), ctypes.POINTER(_PI64)]),
    ("ftn_tensor_leg", _I, [_P, _I, _PI32, ctypes.POINTER(_PI32), ctypes.POINTER(_PI64), _PU8]),
    ("ftn_tensor_data", _I, [_P, _PP]),
    ("ftn_tensor_copy_data", _I, [_P, _P, _P]),
    ("ftn_tensor_cast", _I, [_P, _I, _P, _PP]),
    ("ftn_tensor_scale", _I, [_P, _D, _P, _PP]),
    ("ftn_tensor_axpy", _I, [_D, _P, _P, _P, _PP]),
    ("ftn_tensor_free", _I, [_P]),
    ("ftn_ftranspose", _I, [_P, _PI32, _P, _PP]),
    ("ftn_flip_dual", _I, [_P, _I, _I, _P, _PP]),
    ("ftn_dagger", _I, [_P, _P, _PP]),
    ("ftn_fuse", _I, [_P, _I, _PI32, _I, _I, _P, _PP]),
    ("ftn_ftensordot", _I, [_P, _P, _I, _PI32, _PI32, _I, _I, _P, _PP]),
    ("ftn_ftensordot_noalloc", _I, [_P, _P, _I, _PI32, _PI32, _I, _I, _P, _P, _I64]),
    ("ftn_ftensordot_backward", _I, [_P, _P, _P, _I, _PI32, _PI32, _I, _I, _P, _PP, _PP]),
    ("ftn_compress_bond", _I, [_P, _P, _I, _I, _I64, _D, _I, _P, _PP, _PP, _PD, _PD, _PI64]),
    ("ftn_fuse_backward", _I, [_P, _I, _PI32, _I, _I, _P, _P, _PP]),
    ("ftn_compress_bond_backward", _I, [_P, _P, _I, _I, _I64, _D, _I, _P, _P, _P, _PP, _PP]),
    ("ftn_net_create", _I, [_I, _PP, _I, _PI32, _I, _PI32, _PP]),
    ("ftn_net_free", _I, [_P]),
    ("ftn_contract_network", _I, [_P, _I, _PI32, _I64, _I, _P, _PD, _PI64, _PP, _PI32, _PD]),
    ("ftn_contract_network_grad", _I, [_P, _I, _PI32, _I64, _I, _I, _P, _PD, _PI64, _PP]),
    ("ftn_amplitudes", _I, [_I, _PP, _I, _PI32, _I, _PI32, _I64, _I, _I64, _PI32, _I, _P, _PD, _PI64]),
    ("ftn_autotune", _I, [_I]),
    ("ftn_autotune_load", _I, [ctypes.c_char_p]),
    ("ftn_autotune_save", _I, [ctypes.c_char_p]),
    ("ftn_autotune_stats", _I, [_PI64, _PI64, _PI64]),
    ("ftn_profile_enable", _I, [_I]),
    ("ftn_profile_collect", _I, [_PD, _PD, _PD, _PD]),
    ("ftn_memory_stats", _I, [_I, _PI64, _PI64, _PI64, _I]),
]

PROF_CLASSES = ["gemm_f64", "gemm_f32", "gemm_bf16x3", "permute", "factor", "other",
                # single kernels inside gemm_f64 and factor (also counted there)
                "k_gemm_f64_64x64", "k_gemm_f64_128x128", "k_gemm_f64_256x16", "k_gemm_f64_256x32",
                "k_gemm_f64_16x256", "k_gemm_f64_32x256", "k_splitk_reduce_f64", "k_orth_factor",
                "k_jacobi_sweep", "k_jacobi_sweep_la", "k_jacobi_vectors", "k_svd_cols", "k_skinny_f64", "k_gemm_f64_tall"]
# the classes that are single kernels (the permute class is one kernel template)
PROF_KERNELS = ["gemm_f32", "gemm_bf16x3", "permute"] + PROF_CLASSES[6:]


def profile_enable(on=True):
    load_library()
    _check(_lib.ftn_profile_enable(1 if on else 0))


def profile_collect():
    """{class: (ms, launches, work, algorithmic bytes)} since the last collect."""
    n = len(PROF_CLASSES)
    ms, cnt, wk, by = [(ctypes.c_double * n)() for _ in range(4)]
    _check(_lib.ftn_profile_collect(ms, cnt, wk, by))
    return {c: (ms[i], cnt[i], wk[i], by[i]) for i, c in enumerate(PROF_CLASSES)}


def autotune(mode):
    """GEMM tile autotuner: 0 heuristic, 1 stored choices, 2 tune unseen shapes."""
    load_library()
    _check(_lib.ftn_autotune(int(mode)))


def autotune_load(path):
    load_library()
    _check(_lib.ftn_autotune_load(str(path).encode()))


def autotune_save(path):
    load_library()
    _check(_lib.ftn_autotune_save(str(path).encode()))


def autotune_stats():
    load_library()
    e, t, h = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.ftn_autotune_stats(ctypes.byref(e), ctypes.byref(t), ctypes.byref(h)))
    return dict(entries=e.value, tuned=t.value, hits=h.value)


_ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
_torch_hooks = None


def use_torch_allocator(on=True):
    """Route the library's device allocations through torch's caching allocator
    (on=True) or back to the library's own (on=False). Blocks are always
    returned to the allocator that made them."""
    global _torch_hooks
    load_library()
    if not on:
        _check(_lib.ftn_set_allocator(None, None, None))
        return
    import torch

    def _alloc(size, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(size), stream=int(stream or 0))
        except Exception:  # reported by the library as FTN_ENOMEM
            return None

    def _free(ptr, stream, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    hooks = (_ALLOC_T(_alloc), _FREE_T(_free))
    _check(_lib.ftn_set_allocator(ctypes.cast(hooks[0], ctypes.c_void_p), ctypes.cast(hooks[1], ctypes.c_void_p), None))
    _torch_hooks = hooks  # keep the callbacks alive


def memory_stats(device=0, reset_peak=False):
    """{"in_use", "peak", "reserved"}: bytes of the library's caching
    allocator on ``device`` (see ``ftn_memory_stats``); with ``reset_peak``
    the peak is then reset to the current use (the values returned are
    those before the reset)."""
    load_library()
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.ftn_memory_stats(int(device), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                 1 if reset_peak else 0))
    return {"in_use": a.value, "peak": b.value, "reserved": c.value}


class FtnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_ERRORS.get(code, "E?"), code, msg))
        self.code = code


def load_library(path=LIB_PATH):
    """Load libftn.so and declare every entry point; raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    # torch first: the library then binds to the HIP runtime torch has loaded
    # (the one that owns the device memory and streams it is handed)
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise ImportError("libftn.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise FtnError(rc, _lib.ftn_last_error().decode())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _arr(vals, ctype):
    a = (ctype * max(len(vals), 1))(*vals)
    return a


def _legs_args(sym, legs):
    nsect, charges, dims, duals = [], [], [], []
    for (chs, ds, dual) in legs:
        nsect.append(len(chs))
        for q, d in zip(chs, ds):
            q = tuple(int(x) for x in q)
            charges += [q[0], q[1] if len(q) > 1 else 0]
            dims.append(int(d))
        duals.append(int(dual))
    return (_arr(nsect, ctypes.c_int32), _arr(charges, ctypes.c_int32),
            _arr(dims, ctypes.c_int64), _arr(duals, ctypes.c_uint8))


def _total(total):
    t = tuple(int(x) for x in total)
    return _arr([t[0], t[1] if len(t) > 1 else 0], ctypes.c_int32)


class _DeviceArray:
    """A library buffer exposed through the CUDA array interface; holds the
    tensor wrapper that owns the buffer."""

    def __init__(self, owner, ptr, n, typestr):
        self.owner = owner
        self.__cuda_array_interface__ = {"shape": (int(n),), "typestr": typestr, "data": (int(ptr), False),
                                         "version": 2, "strides": None}


class Tensor:
    """Owning wrapper of an ftn_tensor_t handle."""

    def __init__(self, handle):
        self.h = ctypes.c_void_p(handle) if not isinstance(handle, ctypes.c_void_p) else handle

    def __del__(self):
        try:
            if self.h and self.h.value and _lib is not None:
                _lib.ftn_tensor_free(self.h)
                self.h = ctypes.c_void_p()
        except Exception:
            pass

    # --- construction ----------------------------------------------------
    @classmethod
    def from_dense(cls, sym, legs, total, dense):
        """``legs``: list of (charges, dims, dual); ``dense``: torch cuda tensor."""
        load_library()
        import torch
        if not dense.is_cuda:
            raise ValueError("dense must be a device tensor")
        dense = dense.contiguous()
        dt = F64 if dense.dtype == torch.float64 else F32
        if dense.dtype not in (torch.float64, torch.float32):
            raise ValueError("dense must be float64 or float32")
        ns, ch, dm, du = _legs_args(sym, legs)
        out = ctypes.c_void_p()
        _check(_lib.ftn_tensor_from_dense(sym, dt, len(legs), ns, ch, dm, du, _total(total),
                                          ctypes.c_void_p(dense.data_ptr()), _stream(),
                                          ctypes.byref(out)))
        return cls(out)

    @classmethod
    def create(cls, sym, legs, total, dtype=F64, data=None):
        load_library()
        ns, ch, dm, du = _legs_args(sym, legs)
        out = ctypes.c_void_p()
        src = ctypes.c_void_p(data.data_ptr()) if data is not None else None
        _check(_lib.ftn_tensor_create(sym, dtype, len(legs), ns, ch, dm, du, _total(total), src,
                                      _stream(), ctypes.byref(out)))
        return cls(out)

    @classmethod
    def wrap(cls, sym, legs, total, data):
        """A tensor whose block data are ``data`` (a contiguous device torch
        tensor, float64 or float32), without a copy; ``data`` is kept alive by
        the returned wrapper."""
        load_library()
        if not data.is_contiguous():
            raise ValueError("wrap needs contiguous data")
        ns, ch, dm, du = _legs_args(sym, legs)
        out = ctypes.c_void_p()
        dtype = F64 if data.dtype == __import__("torch").float64 else F32
        _check(_lib.ftn_tensor_wrap(sym, dtype, len(legs), ns, ch, dm, du, _total(total),
                                    ctypes.c_void_p(data.data_ptr()), _stream(), ctypes.byref(out)))
        t = cls(out)
        t._keep = data
        return t

    # --- queries ---------------------------------------------------------
    def info(self):
        sym, dt, nd = _I(), _I(), _I()
        nb, sz = _I64(), _I64()
        tot = (ctypes.c_int32 * 2)()
        _check(_lib.ftn_tensor_info(self.h, ctypes.byref(sym), ctypes.byref(dt), ctypes.byref(nd),
                                    ctypes.byref(nb), ctypes.byref(sz), tot))
        return dict(sym=sym.value, dtype=dt.value, ndim=nd.value, nblocks=nb.value,
                    size=sz.value, total=(tot[0], tot[1]))

    @property
    def ndim(self):
        return self.info()["ndim"]

    @property
    def size(self):
        return self.info()["size"]

    def blocks(self):
        inf = self.info()
        k, o, s = _PI32(), _PI64(), _PI64()
        _check(_lib.ftn_tensor_blocks(self.h, ctypes.byref(k), ctypes.byref(o), ctypes.byref(s)))
        nb, nd = inf["nblocks"], inf["ndim"]
        keys = np.ctypeslib.as_array(k, shape=(nb * nd,)).copy().reshape(nb, nd) if nb * nd else np.zeros((nb, nd), np.int32)
        offs = np.ctypeslib.as_array(o, shape=(nb + 1,)).copy()
        shp = np.ctypeslib.as_array(s, shape=(nb * nd,)).copy().reshape(nb, nd) if nb * nd else np.zeros((nb, nd), np.int64)
        return keys, offs, shp

    def leg(self, i):
        ns = ctypes.c_int32()
        ch, dm = _PI32(), _PI64()
        du = ctypes.c_uint8()
        _check(_lib.ftn_tensor_leg(self.h, i, ctypes.byref(ns), ctypes.byref(ch), ctypes.byref(dm),
                                   ctypes.byref(du)))
        n = ns.value
        c = np.ctypeslib.as_array(ch, shape=(2 * n,)).copy().reshape(n, 2) if n else np.zeros((0, 2), np.int32)
        d = np.ctypeslib.as_array(dm, shape=(n,)).copy() if n else np.zeros(0, np.int64)
        return [tuple(int(x) for x in r) for r in c], [int(x) for x in d], int(du.value)

    def legs(self):
        return [self.leg(i) for i in range(self.ndim)]

    def data(self):
        """Copy of the block data as a torch device tensor."""
        import torch
        inf = self.info()
        dt = torch.float64 if inf["dtype"] == F64 else torch.float32
        out = torch.empty(inf["size"], dtype=dt, device="cuda")
        if inf["size"]:
            _check(_lib.ftn_tensor_copy_data(self.h, ctypes.c_void_p(out.data_ptr()), _stream()))
        return out

    def data_view(self):
        """The block data as a torch device tensor without a copy (the
        library's buffer, kept alive by the returned tensor)."""
        import torch
        inf = self.info()
        dt = torch.float64 if inf["dtype"] == F64 else torch.float32
        if inf["size"] == 0:
            return torch.empty(0, dtype=dt, device="cuda")
        p = ctypes.c_void_p()
        _check(_lib.ftn_tensor_data(self.h, ctypes.byref(p)))
        return torch.as_tensor(_DeviceArray(self, p.value, inf["size"], "<f8" if inf["dtype"] == F64 else "<f4"),
                               device="cuda")

    def to_dense(self):
        import torch
        inf = self.info()
        dt = torch.float64 if inf["dtype"] == F64 else torch.float32
        shape = [sum(l[1]) for l in self.legs()]
        out = torch.empty(shape, dtype=dt, device="cuda")
        _check(_lib.ftn_tensor_to_dense(self.h, ctypes.c_void_p(out.data_ptr()), _stream()))
        return out

    def cast(self, dtype):
        out = ctypes.c_void_p()
        _check(_lib.ftn_tensor_cast(self.h, dtype, _stream(), ctypes.byref(out)))
        return Tensor(out)

    def scale(self, alpha):
        out = ctypes.c_void_p()
        _check(_lib.ftn_tensor_scale(self.h, float(alpha), _stream(), ctypes.byref(out)))
        return Tensor(out)


def axpy(alpha, x, y):
    """alpha * x + y as a new tensor (same structure and dtype)."""
    out = ctypes.c_void_p()
    _check(_lib.ftn_tensor_axpy(float(alpha), x.h, y.h, _stream(), ctypes.byref(out)))
    return Tensor(out)


def ftranspose(a, perm):
    out = ctypes.c_void_p()
    _check(_lib.ftn_ftranspose(a.h, _arr([int(p) for p in perm], ctypes.c_int32), _stream(), ctypes.byref(out)))
    return Tensor(out)


def flip_dual(a, leg, with_sign=-1):
    out = ctypes.c_void_p()
    _check(_lib.ftn_flip_dual(a.h, int(leg), int(with_sign), _stream(), ctypes.byref(out)))
    return Tensor(out)


def dagger(a):
    out = ctypes.c_void_p()
    _check(_lib.ftn_dagger(a.h, _stream(), ctypes.byref(out)))
    return Tensor(out)


def fuse(a, legs, conv=LOCAL, rev=0):
    out = ctypes.c_void_p()
    _check(_lib.ftn_fuse(a.h, len(legs), _arr([int(l) for l in legs], ctypes.c_int32), int(conv), int(rev),
                         _stream(), ctypes.byref(out)))
    return Tensor(out)


def fuse_backward(a, legs, dout, conv=LOCAL, rev=0):
    """Cotangent of a for the cotangent dout of fuse(a, legs, conv, rev)."""
    out = ctypes.c_void_p()
    _check(_lib.ftn_fuse_backward(a.h, len(legs), _arr([int(l) for l in legs], ctypes.c_int32), int(conv), int(rev),
                                  dout.h, _stream(), ctypes.byref(out)))
    return Tensor(out)


def ftensordot(a, b, axes_a, axes_b, conv=LOCAL, gemm=GEMM_F64):
    out = ctypes.c_void_p()
    _check(_lib.ftn_ftensordot(a.h, b.h, len(axes_a), _arr([int(x) for x in axes_a], ctypes.c_int32),
                               _arr([int(x) for x in axes_b], ctypes.c_int32), int(conv), int(gemm),
                               _stream(), ctypes.byref(out)))
    return Tensor(out)


def ftensordot_noalloc(a, b, axes_a, axes_b, out, conv=LOCAL, gemm=GEMM_F64):
    """ftensordot into ``out`` (a contiguous device tensor of the output's size
    and dtype) without any device allocation; needs a cached plan."""
    _check(_lib.ftn_ftensordot_noalloc(a.h, b.h, len(axes_a), _arr([int(x) for x in axes_a], ctypes.c_int32),
                                       _arr([int(x) for x in axes_b], ctypes.c_int32), int(conv), int(gemm),
                                       _stream(), ctypes.c_void_p(out.data_ptr()), int(out.numel())))
    return out


def ftensordot_backward(a, b, dc, axes_a, axes_b, conv=LOCAL, gemm=GEMM_F64):
    """Adjoint of ftensordot: (dA, dB) for the cotangent dC of its output."""
    da, db = ctypes.c_void_p(), ctypes.c_void_p()
    _check(_lib.ftn_ftensordot_backward(a.h, b.h, dc.h, len(axes_a), _arr([int(x) for x in axes_a], ctypes.c_int32),
                                        _arr([int(x) for x in axes_b], ctypes.c_int32), int(conv), int(gemm),
                                        _stream(), ctypes.byref(da), ctypes.byref(db)))
    return Tensor(da), Tensor(db)


def compress_bond(a, b, leg_a, leg_b, chi, cutoff=1e-12, conv=LOCAL):
    ao, bo = ctypes.c_void_p(), ctypes.c_void_p()
    disc = ctypes.c_double()
    sv = (ctypes.c_double * int(chi))()
    nk = ctypes.c_int64()
    _check(_lib.ftn_compress_bond(a.h, b.h, int(leg_a), int(leg_b), int(chi), float(cutoff), int(conv),
                                  _stream(), ctypes.byref(ao), ctypes.byref(bo), ctypes.byref(disc), sv,
                                  ctypes.byref(nk)))
    return Tensor(ao), Tensor(bo), dict(discarded=disc.value, svals=list(sv[:nk.value]))


def compress_bond_backward(a, b, leg_a, leg_b, chi, da_out, db_out, cutoff=1e-12, conv=LOCAL):
    """Cotangents (da, db) of compress_bond for cotangents of its outputs."""
    da, db = ctypes.c_void_p(), ctypes.c_void_p()
    _check(_lib.ftn_compress_bond_backward(a.h, b.h, int(leg_a), int(leg_b), int(chi), float(cutoff), int(conv),
                                           da_out.h, db_out.h, _stream(), ctypes.byref(da), ctypes.byref(db)))
    return Tensor(da), Tensor(db)


class Network:
    def __init__(self, tensors, bonds, conv=LOCAL, positions=None):
        load_library()
        self.tensors = list(tensors)  # keep the wrappers alive
        hs = (ctypes.c_void_p * len(tensors))(*[t.h.value for t in tensors])
        ends = []
        for b in bonds:
            ends += [int(x) for x in b]
        pos = _arr([int(p) for p in positions], ctypes.c_int32) if positions is not None else None
        self.h = ctypes.c_void_p()
        _check(_lib.ftn_net_create(len(tensors), hs, len(bonds), _arr(ends, ctypes.c_int32), int(conv), pos,
                                   ctypes.byref(self.h)))

    def __del__(self):
        try:
            if self.h and self.h.value and _lib is not None:
                _lib.ftn_net_free(self.h)
        except Exception:
            pass

    def contract(self, path, chi=0, gemm=GEMM_F64, open_legs=False):
        """Returns (mantissa, exp2, stats) or (tensor, exp2, leg_src, stats)."""
        flat = []
        for (i, j) in path:
            flat += [int(i), int(j)]
        m = ctypes.c_double()
        e = ctypes.c_int64()
        st = (ctypes.c_double * 8)()
        out = ctypes.c_void_p()
        src = (ctypes.c_int32 * 64)()
        _check(_lib.ftn_contract_network(self.h, len(path), _arr(flat, ctypes.c_int32), int(chi or 0), int(gemm),
                                         _stream(), ctypes.byref(m), ctypes.byref(e),
                                         ctypes.byref(out) if open_legs else None, src, st))
        stats = dict(flops=st[0], compressions=int(st[1]), discarded=st[2], near_ties=int(st[3]),
                     max_entries=st[4], compress_textbook_flops=st[5])
        if open_legs and out.value:
            t = Tensor(out)
            n = t.ndim
            return t, e.value, [(src[2 * k], src[2 * k + 1]) for k in range(n)], stats
        return m.value, e.value, stats


def _network_grad(self, path, chi=0, checkpoint=0, gemm=GEMM_F64):
    """(mantissa, exp2, grads) of a closed network: value = m * 2**e and
    grads[t] = d(value)/d(tensor t) * 2**-e, computed by the library's
    backward pass (checkpoint: path steps per recomputation segment, 0 keeps
    every intermediate)."""
    flat = []
    for (i, j) in path:
        flat += [int(i), int(j)]
    m = ctypes.c_double()
    e = ctypes.c_int64()
    n = len(self.tensors)
    gh = (ctypes.c_void_p * n)()
    _check(_lib.ftn_contract_network_grad(self.h, len(path), _arr(flat, ctypes.c_int32), int(chi or 0), int(gemm),
                                          int(checkpoint), _stream(), ctypes.byref(m), ctypes.byref(e), gh))
    return m.value, e.value, [Tensor(ctypes.c_void_p(gh[t])) for t in range(n)]


Network.contract_grad = _network_grad


def amplitudes(sites, bonds, path, configs, chi=0, gemm=GEMM_F64, nworkers=8):
    """<n|psi> for every row of ``configs`` (physical index per site).

    ``sites``: Tensors with the physical leg first, in global (site) order;
    ``bonds``: (site, leg, site, leg) with legs >= 1; ``path``: SSA pairs over
    the sites. Returns (mantissa, exp2) numpy arrays: amplitude = m * 2**e.
    """
    load_library()
    cfg = np.ascontiguousarray(np.asarray(configs, dtype=np.int32))
    if cfg.ndim != 2 or cfg.shape[1] != len(sites):
        raise ValueError("configs must be (nsamples, nsites)")
    ns = cfg.shape[0]
    hs = (ctypes.c_void_p * len(sites))(*[t.h.value for t in sites])
    ends = []
    for b in bonds:
        ends += [int(x) for x in b]
    flat = []
    for (i, j) in path:
        flat += [int(i), int(j)]
    m = np.zeros(ns, dtype=np.float64)
    e = np.zeros(ns, dtype=np.int64)
    _check(_lib.ftn_amplitudes(len(sites), hs, len(bonds), _arr(ends, ctypes.c_int32), len(path),
                               _arr(flat, ctypes.c_int32), int(chi or 0), int(gemm), ns,
                               cfg.ctypes.data_as(_PI32), int(nworkers), _stream(),
                               m.ctypes.data_as(_PD), e.ctypes.data_as(_PI64)))
    return m, e
