"""ctypes binding of libdd (argument marshalling only).

Every computation runs in the HIP library ``libdd.so`` next to this file;
nothing here computes on the host.  Importing this module fails loudly when
the library has not been built.  Function names follow the C ABI in
``include/dd.h`` without the ``dd_`` prefix.

Device buffers are torch tensors on the GPU (complex128 for spinors and
links, float64 for actions); the library orders its work after the current
torch stream and synchronises before returning.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdd.so")

DD_OK, DD_EINVAL, DD_ENOMEM, DD_EDEVICE, DD_ENOCONV, DD_EUNSUPPORTED = range(6)
F64, F32, BF16 = 0, 1, 2
BICGSTAB, GMRES = 0, 1
KCLASS_HOP_F64, KCLASS_HOP_F32, KCLASS_HOP_BF16, KCLASS_GMRES, KCLASS_NN_BF16 = 0, 1, 2, 3, 4
KCLASS_DHAT_F32, KCLASS_DHAT_BF16 = 5, 6
TUNE_RHS_GROUP_F64, TUNE_RHS_GROUP_F32, TUNE_HOP_LDS = 0, 1, 2
TUNE_GMRES_THREADS, TUNE_GMRES_QUEUES, TUNE_GMRES_WG_PER_CU, TUNE_MB_FIELDS, TUNE_NN_KERNEL = 3, 4, 5, 6, 7
TUNE_HOP_WALK, TUNE_GMRES_REORTH, TUNE_BICG_FUSE, TUNE_DHAT_WALK, TUNE_DHAT_RHS = 8, 9, 10, 11, 12
_PREC = {"f64": F64, "f32": F32, "bf16": BF16, F64: F64, F32: F32, BF16: BF16}

if not os.path.exists(LIB_PATH):
    raise ImportError("libdd.so is not built; run `python -m paper_2211_06902_amd.build` "
                      "(or __graft_entry__.build())")

# torch must load its HIP runtime first: libdd then binds to that same runtime
# (same SONAME), so torch's device pointers and streams are valid in libdd.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)


def _hip_runtimes():
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    paths.add(os.path.realpath(line.split()[-1]))
    except OSError:
        pass
    return paths


if len(_hip_runtimes()) > 1:
    raise ImportError("two HIP runtimes are mapped (%s); import torch before anything that loads "
                      "libamdhip64" % ", ".join(sorted(_hip_runtimes())))
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double
_PP = ctypes.POINTER(ctypes.c_void_p)


class SolveParams(ctypes.Structure):
    _fields_ = [
        ("tol", _D),
        ("method", _I32),
        ("restart", _I32),
        ("inner_prec", _I32),
        ("inner_tol", _D),
        ("max_outer", _I32),
        ("max_inner", _I32),
        ("check_every", _I32),
        ("use_graph", _I32),
        ("precond", _P),
        ("precond_cycles", _I32),
        ("recover", _I32),
        ("x0", _I32),
    ]


class BicgTuneResult(ctypes.Structure):
    _fields_ = [("rhs_group", _I32), ("dhat_walk", _I32), ("dhat_rhs", _I32), ("bicg_fuse", _I32), ("ms", _D)]


class SolveStats(ctypes.Structure):
    _fields_ = [
        ("iters", _P),
        ("true_relres", _P),
        ("flags", _P),
        ("seconds", _D),
        ("outer_cycles", _I32),
        ("inner_iterations", _I64),
        ("rhs_per_solve", _I32),
        ("resolved_pairs", _I32),
    ]


class TuneResult(ctypes.Structure):
    _fields_ = [
        ("threads", _I32),
        ("queues", _I32),
        ("wg_per_cu", _I32),
        ("ms", _D),
    ]


class NnTrainParams(ctypes.Structure):
    _fields_ = [
        ("epochs", _I32),
        ("batch", _I32),
        ("lr", _D),
        ("beta1", _D),
        ("beta2", _D),
        ("eps", _D),
        ("seed", ctypes.c_uint64),
        ("mask_even", _I32),
    ]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("dd_version", ctypes.c_char_p, [])
_sig("dd_create", _I32, [ctypes.c_int, _P, _PP])
_sig("dd_destroy", _I32, [_P])
_sig("dd_last_error", ctypes.c_char_p, [_P])
_sig("dd_make_blocks", _I32, [_P, _P, _I32, _P, _P, _P, _I32, _PP])
_sig("dd_make_blocks_paper", _I32, [_P, _P, _I32, _P, _PP])
_sig("dd_make_blocks_boxes", _I32, [_P, _P, _I32, _I32, _P, _P, _PP])
_sig("dd_make_frames", _I32, [_P, _P, _PP])
_sig("dd_make_inactive", _I32, [_P, _P, _PP])
_sig("dd_blocks_dpi1", _I32, [_P, _P, _P])
_sig("dd_free_blocks", _I32, [_P])
_sig("dd_blocks_query", _I32, [_P, _P, _P, _P, _P])
_sig("dd_blocks_tables", _I32, [_P, _P, _P, _P, _P])
_sig("dd_blocks_exterior", _I32, [_P, _P, _P, _P, _P, _P])
_sig("dd_load_gauge", _I32, [_P, _P, _P, _I32, _PP])
_sig("dd_free_gauge", _I32, [_P])
_sig("dd_gauge_export", _I32, [_P, _P, _I32, _P])
_sig("dd_gauge_set_clover", _I32, [_P, _P, _P, _D, _D])
_sig("dd_apply_D_block", _I32, [_P, _P, _P, _D, _I32, _P, _P, _I32])
_sig("dd_apply_D_block_noalloc", _I32, [_P, _P, _P, _D, _I32, _P, _P, _I32])
_sig("dd_solve_params_default", None, [ctypes.POINTER(SolveParams)])
_sig("dd_block_solve", _I32, [_P, _P, _P, _D, _P, _P, _I32, ctypes.POINTER(SolveParams),
                              ctypes.POINTER(SolveStats)])
_sig("dd_multiboson_action", _I32, [_P, _P, _P, _D, _I32, _P, _P, _P, ctypes.POINTER(SolveParams), _P, _P,
                                    ctypes.POINTER(SolveStats)])
_sig("dd_tune_set", _I32, [_P, _I32, _I32])
_sig("dd_mb_roots", _I32, [_I32, _D, _P])
_sig("dd_block_logdet", _I32, [_P, _P, _P, _D, _P, _P])
_sig("dd_mb_exterior_source", _I32, [_P, _P, _P, _D, _I32, _P, _P, _I32])
_sig("dd_mb_global_action", _I32, [_P, _P, _P, _D, _I32, _P, _P, ctypes.POINTER(SolveParams), _P, _P,
                                 ctypes.POINTER(SolveStats)])
_sig("dd_mb_apply_W", _I32, [_P, _P, _P, _P, _P, _D, _I32, _P, _P, _P, ctypes.POINTER(SolveParams),
                           ctypes.POINTER(SolveStats)])
_sig("dd_mb_generate", _I32, [_P, _P, _P, _P, _P, _D, _I32, _P, _P, _P, _D, _I32, ctypes.POINTER(SolveParams),
                            _P, _P, ctypes.POINTER(SolveStats)])
_sig("dd_mb_log_reweight", _I32, [_P, _P, _P, _P, _P, _D, _I32, _D, _I32, _I32, _P, ctypes.POINTER(SolveParams),
                                _P, _P, ctypes.POINTER(SolveStats)])
_sig("dd_nn_num_weights", _I64, [])
_sig("dd_nn_create", _I32, [_P, _P, _I32, _P, _PP])
_sig("dd_nn_free", _I32, [_P])
_sig("dd_nn_get_weights", _I32, [_P, _P, _P])
_sig("dd_nn_apply", _I32, [_P, _P, _I32, _P, _P, _I64])
_sig("dd_nn_set_inference", _I32, [_P, _P, _I32])
_sig("dd_nn_apply_blocks", _I32, [_P, _P, _P, _P, _P, _I32])
_sig("dd_nn_train_params_default", None, [ctypes.POINTER(NnTrainParams)])
_sig("dd_nn_loss_grad", _I32, [_P, _P, _P, _P, _P, _I32, _P, _I32, _I32, _P, _P])
_sig("dd_nn_train", _I32, [_P, _P, _P, _P, _P, _I32, _P, _P, _I32, ctypes.POINTER(NnTrainParams), _P, _P])
_sig("dd_autotune_gmres", _I32, [_P, _P, _P, _D, _P, _P, _I32, ctypes.POINTER(SolveParams),
                                 ctypes.POINTER(TuneResult), _I32, _P])
_sig("dd_autotune_bicgstab", _I32, [_P, _P, _P, _D, _P, _P, _I32, ctypes.POINTER(SolveParams), ctypes.c_char_p,
                                   _P, _I32, _P, _P])
_sig("dd_timer_enable", _I32, [_P, _I32])
_sig("dd_timer_reset", _I32, [_P])
_sig("dd_timer_read", _I32, [_P, _I32, _P, _P, _P])


class DDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("libdd status %d: %s" % (status, msg))
        self.status = status


def version() -> str:
    return _lib.dd_version().decode()


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_P)


def _dev(t, dtype_name):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a GPU torch tensor")
    if str(t.dtype) != dtype_name:
        raise TypeError("expected dtype %s, got %s" % (dtype_name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return _P(t.data_ptr())


NN_LINEAR, NN_RELU = 0, 1


def nn_train_params(**kw) -> NnTrainParams:
    p = NnTrainParams()
    _lib.dd_nn_train_params_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def mb_roots(N: int, c: float) -> np.ndarray:
    """u_k, k = 1 .. N/2 (complex), from the library."""
    out = np.zeros(N, dtype=np.float64)
    st = _lib.dd_mb_roots(int(N), float(c), out.ctypes.data_as(_P))
    if st != DD_OK:
        raise DDError(st, "invalid N or c")
    return out[0::2] + 1j * out[1::2]


def nn_num_weights() -> int:
    return int(_lib.dd_nn_num_weights())


def solve_params(**kw) -> SolveParams:
    p = SolveParams()
    _lib.dd_solve_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if k == "inner_prec":
            v = _PREC[v]
        if k == "precond" and isinstance(v, Net):
            v = v._h
        setattr(p, k, v)
    return p


class Net:
    """The learned block preconditioner (FP32 weights and Adam state on the GPU)."""

    def __init__(self, handle, ctx, extent, act):
        self._h = handle
        self._ctx = ctx
        self.extent = extent
        self.act = act
        self.sites = int(np.prod(extent))

    def close(self):
        if self._h:
            _lib.dd_nn_free(self._h)
            self._h = None

    def weights(self):
        w = np.zeros(nn_num_weights(), dtype=np.float32)
        self._ctx._check(_lib.dd_nn_get_weights(self._ctx._h, self._h, w.ctypes.data_as(_P)))
        return w

    def apply(self, x, prec="f32"):
        """x: GPU float32 [n, S, 24] rows -> N(x) of the same shape (prec "f32" or "bf16")."""
        import torch

        y = torch.empty_like(x)
        n = x.numel() // (self.sites * 24)
        self._ctx._check(_lib.dd_nn_apply(self._ctx._h, self._h, _PREC[prec], _dev(x, "torch.float32"),
                                          _dev(y, "torch.float32"), n))
        return y

    def apply_blocks(self, blocks, x, n_rhs=None):
        """The network as a solve applies it: x [n_rhs, total_sites, 4, 3] complex128 on the GPU (solver
        layout) -> N of its even sites on the even sites (odd sites zero), same shape."""
        import torch

        if n_rhs is None:
            n_rhs = x.numel() // (blocks.total_sites * 12)
        y = torch.empty_like(x)
        self._ctx._check(_lib.dd_nn_apply_blocks(self._ctx._h, self._h, blocks._h, _dev(x, "torch.complex128"),
                                                 _dev(y, "torch.complex128"), int(n_rhs)))
        return y

    def set_inference(self, prec):
        """Precision of the network inside solves: "bf16" (default) or "f32"."""
        self._ctx._check(_lib.dd_nn_set_inference(self._ctx._h, self._h, _PREC[prec]))

    def loss_grad(self, blocks, src, sol, n_rhs, pairs, mask_even=1):
        pr = _i32(pairs)
        loss = _D()
        g = np.zeros(nn_num_weights(), dtype=np.float32)
        self._ctx._check(_lib.dd_nn_loss_grad(self._ctx._h, self._h, blocks._h, _dev(src, "torch.complex128"),
                                              _dev(sol, "torch.complex128"), int(n_rhs), pr.ctypes.data_as(_P),
                                              int(pr.size), int(mask_even), ctypes.byref(loss), g.ctypes.data_as(_P)))
        return loss.value, g

    def train(self, blocks, src, sol, n_rhs, val_src=None, val_sol=None, val_n_rhs=0, params=None):
        p = params if params is not None else nn_train_params()
        tl = np.zeros(p.epochs)
        vl = np.zeros(p.epochs)
        vs = _dev(val_src, "torch.complex128") if val_src is not None else None
        vo = _dev(val_sol, "torch.complex128") if val_sol is not None else None
        self._ctx._check(_lib.dd_nn_train(self._ctx._h, self._h, blocks._h, _dev(src, "torch.complex128"),
                                          _dev(sol, "torch.complex128"), int(n_rhs), vs, vo, int(val_n_rhs),
                                          ctypes.byref(p), tl.ctypes.data_as(_P), vl.ctypes.data_as(_P)))
        return tl, vl


class Blocks:
    """A block decomposition (boxes, even-odd maps, neighbour tables)."""

    def __init__(self, handle, ctx):
        self._h = handle
        self._ctx = ctx
        nb, ts, tb, il = _I64(), _I64(), _I64(), _I64()
        _lib.dd_blocks_query(self._h, ctypes.byref(nb), ctypes.byref(ts), ctypes.byref(tb), ctypes.byref(il))
        self.n_blocks, self.total_sites, self.total_bnd_sites, self.inner_links = nb.value, ts.value, tb.value, il.value

    def tables(self):
        """(boxes[nb,16], sites[total], eo[total], bnd[total_bnd]) as numpy arrays."""
        boxes = np.zeros((self.n_blocks, 16), dtype=np.int32)
        sites = np.zeros(self.total_sites, dtype=np.int64)
        eo = np.zeros(self.total_sites, dtype=np.int32)
        bnd = np.zeros(max(self.total_bnd_sites, 1), dtype=np.int32)
        _lib.dd_blocks_tables(self._h, _ptr(boxes), _ptr(sites), _ptr(eo), _ptr(bnd))
        return boxes, sites, eo, bnd[: self.total_bnd_sites]

    def exterior(self):
        """Exterior hops of the multi-boson source: (block, site, code, nbr) arrays, one entry per hop."""
        n = _I64()
        _lib.dd_blocks_exterior(self._h, ctypes.byref(n), None, None, None, None)
        blk = np.zeros(n.value, dtype=np.int32)
        site = np.zeros(n.value, dtype=np.int32)
        code = np.zeros(n.value, dtype=np.int32)
        nbr = np.zeros(n.value, dtype=np.int64)
        if n.value:
            _lib.dd_blocks_exterior(self._h, ctypes.byref(n), _ptr(blk), _ptr(site), _ptr(code), _ptr(nbr))
        return blk, site, code, nbr

    def dpi1(self):
        """dPi_1 sites of an inactive-region domain (global canonical indices, ascending)."""
        n = _I64()
        st = _lib.dd_blocks_dpi1(self._h, ctypes.byref(n), None)
        if st != DD_OK:
            raise DDError(st, _lib.dd_last_error(None).decode())
        out = np.zeros(n.value, dtype=np.int64)
        if n.value:
            _lib.dd_blocks_dpi1(self._h, ctypes.byref(n), _ptr(out))
        return out

    def close(self):
        if self._h:
            _lib.dd_free_blocks(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _make(fn, ctx, *args):
    out = _P()
    st = fn(ctx._h if ctx is not None else None, *args, ctypes.byref(out))
    if st != DD_OK:
        msg = _lib.dd_last_error(ctx._h if ctx is not None else None).decode()
        raise DDError(st, msg)
    return Blocks(out, ctx)


def make_blocks(ctx, L, time_bc, segs, shift=(0, 0, 0, 0), inner_d=0) -> Blocks:
    """Tile decomposition; ctx None builds host tables only."""
    nseg = _i32([len(s) for s in segs])
    seg = _i32([v for s in segs for v in s])
    return _make(_lib.dd_make_blocks, ctx, _ptr(_i32(L)), int(time_bc), _ptr(seg), _ptr(nseg), _ptr(_i32(shift)),
                 int(inner_d))


def make_blocks_paper(ctx, L, time_bc, bd) -> Blocks:
    return _make(_lib.dd_make_blocks_paper, ctx, _ptr(_i32(L)), int(time_bc), _ptr(_i32(bd)))


def make_frames(ctx, blocks) -> Blocks:
    """The frames (box minus inner box) of `blocks` as solve domains."""
    return _make(_lib.dd_make_frames, ctx, blocks._h)


def make_inactive(ctx, blocks) -> Blocks:
    """The inactive region (the lattice minus the inner boxes of `blocks`) as one solve domain."""
    return _make(_lib.dd_make_inactive, ctx, blocks._h)


def make_blocks_boxes(ctx, L, time_bc, boxes, inner=None) -> Blocks:
    b = _i32(boxes)
    inn = _i32(inner) if inner is not None else None
    return _make(_lib.dd_make_blocks_boxes, ctx, _ptr(_i32(L)), int(time_bc), int(b.size // 8), _ptr(b),
                 _ptr(inn) if inn is not None else None)


class Gauge:
    def __init__(self, handle, ctx, blocks, low):
        self._h = handle
        self._ctx = ctx
        self.blocks = blocks
        self.low = low

    def export(self, prec):
        """Packed links (rows 0 and 1 of each link) of precision prec as a GPU tensor (float64, float32 or
        int16 bits)."""
        import torch

        n = self.blocks.total_sites * 48
        dt = {F64: torch.float64, F32: torch.float32, BF16: torch.int16}[_PREC[prec]]
        out = torch.empty(n, dtype=dt, device="cuda")
        self._ctx._check(_lib.dd_gauge_export(self._ctx._h, self._h, _PREC[prec], _P(out.data_ptr())))
        return out

    def set_clover(self, U, kappa, csw):
        """The clover term for this gauge's operator from the global FP64 field U [V, 4, 3, 3]
        (c_sw = 0: back to the Wilson operator); later operators and solves must use this kappa."""
        self._ctx._check(_lib.dd_gauge_set_clover(self._ctx._h, self._h, _dev(U, "torch.complex128") if csw else None,
                                                  float(kappa), float(csw)))
        return self

    def close(self):
        if self._h:
            _lib.dd_free_gauge(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """A libdd context on one GPU; work is ordered after torch's current stream."""

    def __init__(self, device: int = 0):
        import torch

        torch.cuda.init()
        stream = torch.cuda.current_stream(device).cuda_stream
        h = _P()
        st = _lib.dd_create(int(device), _P(stream), ctypes.byref(h))
        if st != DD_OK:
            raise DDError(st, "dd_create failed on device %d" % device)
        self._h = h
        self.device = device

    def _check(self, st, allow=()):
        if st != DD_OK and st not in allow:
            raise DDError(st, _lib.dd_last_error(self._h).decode())
        return st

    def close(self):
        if self._h:
            _lib.dd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # geometry
    def make_blocks(self, L, time_bc, segs, shift=(0, 0, 0, 0), inner_d=0) -> Blocks:
        return make_blocks(self, L, time_bc, segs, shift, inner_d)

    def make_blocks_paper(self, L, time_bc, bd) -> Blocks:
        return make_blocks_paper(self, L, time_bc, bd)

    def make_blocks_boxes(self, L, time_bc, boxes, inner=None) -> Blocks:
        return make_blocks_boxes(self, L, time_bc, boxes, inner)

    def make_frames(self, blocks) -> Blocks:
        return make_frames(self, blocks)

    def make_inactive(self, blocks) -> Blocks:
        return make_inactive(self, blocks)

    # gauge
    def load_gauge(self, blocks: Blocks, U, low_prec="f32") -> Gauge:
        out = _P()
        self._check(_lib.dd_load_gauge(self._h, blocks._h, _dev(U, "torch.complex128"), _PREC[low_prec],
                                       ctypes.byref(out)))
        return Gauge(out, self, blocks, _PREC[low_prec])

    # operator
    def apply_D_block(self, blocks: Blocks, gauge: Gauge, kappa, prec, x, y=None, n_rhs=None):
        import torch

        if n_rhs is None:
            n_rhs = x.numel() // (blocks.total_sites * 12)
        if y is None:
            y = torch.empty_like(x)
        self._check(_lib.dd_apply_D_block(self._h, blocks._h, gauge._h, float(kappa), _PREC[prec],
                                          _dev(x, "torch.complex128"), _dev(y, "torch.complex128"), int(n_rhs)))
        return y

    def apply_D_block_noalloc(self, blocks: Blocks, gauge: Gauge, kappa, prec, x, y, n_rhs=None):
        """y = D_Lambda x into the caller's y, with the library's preallocated per-device scratch
        (no device allocation by the library)."""
        if n_rhs is None:
            n_rhs = x.numel() // (blocks.total_sites * 12)
        self._check(_lib.dd_apply_D_block_noalloc(self._h, blocks._h, gauge._h, float(kappa), _PREC[prec],
                                                  _dev(x, "torch.complex128"), _dev(y, "torch.complex128"),
                                                  int(n_rhs)))
        return y

    # solves
    def block_solve(self, blocks: Blocks, gauge: Gauge, kappa, b, x=None, n_rhs=None, params=None):
        """Returns (x, stats dict, status) with status DD_OK or DD_ENOCONV."""
        import torch

        if n_rhs is None:
            n_rhs = b.numel() // (blocks.total_sites * 12)
        if x is None:
            x = torch.empty_like(b)
        if params is None:
            params = solve_params()
        np_ = n_rhs * blocks.n_blocks
        iters = np.zeros(np_, dtype=np.int32)
        rel = np.zeros(np_, dtype=np.float64)
        flags = np.zeros(np_, dtype=np.int32)
        stats = SolveStats(_ptr(iters), _ptr(rel), _ptr(flags), 0.0, 0, 0, 0, 0)
        st = self._check(_lib.dd_block_solve(self._h, blocks._h, gauge._h, float(kappa), _dev(b, "torch.complex128"),
                                             _dev(x, "torch.complex128"), int(n_rhs), ctypes.byref(params),
                                             ctypes.byref(stats)), allow=(DD_ENOCONV,))
        info = {"iters": iters.reshape(n_rhs, blocks.n_blocks), "true_relres": rel.reshape(n_rhs, blocks.n_blocks),
                "flags": flags.reshape(n_rhs, blocks.n_blocks), "seconds": stats.seconds,
                "outer_cycles": stats.outer_cycles, "inner_iterations": stats.inner_iterations,
                "rhs_per_solve": stats.rhs_per_solve, "resolved_pairs": stats.resolved_pairs}
        return x, info, st

    def multiboson_action(self, blocks: Blocks, gauge: Gauge, kappa, u, chi, xi, params=None, S_block=None):
        """Returns (S_block tensor [n_blocks] float64, S_total, stats dict, status)."""
        import torch

        u = np.ascontiguousarray(np.asarray(u, dtype=np.complex128).reshape(-1))
        nf = u.size
        uu = np.ascontiguousarray(np.stack([u.real, u.imag], axis=1).reshape(-1))
        if S_block is None:
            S_block = torch.empty(blocks.n_blocks, dtype=torch.float64, device="cuda")
        if params is None:
            params = solve_params()
        np_ = nf * blocks.n_blocks
        iters = np.zeros(np_, dtype=np.int32)
        rel = np.zeros(np_, dtype=np.float64)
        flags = np.zeros(np_, dtype=np.int32)
        stats = SolveStats(_ptr(iters), _ptr(rel), _ptr(flags), 0.0, 0, 0, 0, 0)
        tot = _D()
        st = self._check(_lib.dd_multiboson_action(self._h, blocks._h, gauge._h, float(kappa), int(nf), _ptr(uu),
                                                   _dev(chi, "torch.complex128"), _dev(xi, "torch.complex128"),
                                                   ctypes.byref(params), _dev(S_block, "torch.float64"),
                                                   ctypes.byref(tot), ctypes.byref(stats)), allow=(DD_ENOCONV,))
        info = {"iters": iters.reshape(nf, blocks.n_blocks), "true_relres": rel.reshape(nf, blocks.n_blocks),
                "flags": flags.reshape(nf, blocks.n_blocks), "seconds": stats.seconds,
                "outer_cycles": stats.outer_cycles, "rhs_per_solve": stats.rhs_per_solve,
                "resolved_pairs": stats.resolved_pairs}
        return S_block, tot.value, info, st

    def block_logdet(self, blocks: Blocks, gauge: Gauge, kappa):
        """Per-block ln det D_Lambda (FP64): (numpy [n_blocks] complex ln|det| + i phase, total)."""
        import torch

        out = torch.empty((blocks.n_blocks, 2), dtype=torch.float64, device="cuda")
        tot = (ctypes.c_double * 2)()
        self._check(_lib.dd_block_logdet(self._h, blocks._h, gauge._h, float(kappa), _dev(out, "torch.float64"), tot))
        o = out.cpu().numpy()
        return o[:, 0] + 1j * o[:, 1], complex(tot[0], tot[1])

    def mb_global_action(self, domain: Blocks, gauge: Gauge, kappa, u, chi_global, params=None):
        """Global rest S^r_MB per field on an inactive-region domain: (S per field [n_fields] numpy, total,
        stats dict, status).  chi_global [n_fields, V, 4, 3] complex128 on the GPU."""
        u = np.ascontiguousarray(np.asarray(u, dtype=np.complex128).reshape(-1))
        nf = u.size
        uu = np.ascontiguousarray(np.stack([u.real, u.imag], axis=1).reshape(-1))
        if params is None:
            params = solve_params()
        iters = np.zeros(nf, dtype=np.int32)
        rel = np.zeros(nf, dtype=np.float64)
        flags = np.zeros(nf, dtype=np.int32)
        stats = SolveStats(_ptr(iters), _ptr(rel), _ptr(flags), 0.0, 0, 0, 0, 0)
        Sf = np.zeros(nf, dtype=np.float64)
        tot = _D()
        st = self._check(_lib.dd_mb_global_action(self._h, domain._h, gauge._h, float(kappa), int(nf), _ptr(uu),
                                                   _dev(chi_global, "torch.complex128"), ctypes.byref(params),
                                                   _ptr(Sf), ctypes.byref(tot), ctypes.byref(stats)),
                         allow=(DD_ENOCONV,))
        info = {"iters": iters, "true_relres": rel, "flags": flags, "seconds": stats.seconds,
                "outer_cycles": stats.outer_cycles, "rhs_per_solve": stats.rhs_per_solve}
        return Sf, tot.value, info, st

    @staticmethod
    def _cplx_pairs(z):
        z = np.ascontiguousarray(np.asarray(z, dtype=np.complex128).reshape(-1))
        return z.size, np.ascontiguousarray(np.stack([z.real, z.imag], axis=1).reshape(-1))

    @staticmethod
    def _wstats(stats):
        return {"seconds": stats.seconds, "outer_cycles": stats.outer_cycles,
                "inner_iterations": stats.inner_iterations, "rhs_per_solve": stats.rhs_per_solve}

    def mb_apply_W(self, blocks: Blocks, gauge: Gauge, domain: Blocks, domain_gauge: Gauge, kappa, z, chi_global,
                   out=None, params=None):
        """W_z chi on dPi (eq. MBaction), one z per field: (out [n_fields, V, 4, 3] complex128 on the GPU,
        info, status).  domain = make_inactive(blocks), domain_gauge its gauge (same links)."""
        import torch

        nf, zz = self._cplx_pairs(z)
        if out is None:
            out = torch.empty_like(chi_global)
        if params is None:
            params = solve_params()
        stats = SolveStats(None, None, None, 0.0, 0, 0, 0, 0)
        st = self._check(_lib.dd_mb_apply_W(self._h, blocks._h, gauge._h, domain._h, domain_gauge._h, float(kappa),
                                            int(nf), _ptr(zz), _dev(chi_global, "torch.complex128"),
                                            _dev(out, "torch.complex128"), ctypes.byref(params),
                                            ctypes.byref(stats)), allow=(DD_ENOCONV,))
        return out, self._wstats(stats), st

    def mb_generate(self, blocks: Blocks, gauge: Gauge, domain: Blocks, domain_gauge: Gauge, kappa, u, eta_global,
                    tol=1e-10, maxit=100, params=None, chi=None):
        """chi_k = W_{u_k}^{-1} eta_k on dPi (the multi-boson fields from the caller's Gaussian noise):
        (chi [n_fields, V, 4, 3] on the GPU, iterations [n_fields], true relres [n_fields], info, status)."""
        import torch

        nf, uu = self._cplx_pairs(u)
        if chi is None:
            chi = torch.empty_like(eta_global)
        if params is None:
            params = solve_params(tol=min(1e-12, tol * 1e-2))
        its = np.zeros(nf, dtype=np.int32)
        rel = np.zeros(nf, dtype=np.float64)
        stats = SolveStats(None, None, None, 0.0, 0, 0, 0, 0)
        st = self._check(_lib.dd_mb_generate(self._h, blocks._h, gauge._h, domain._h, domain_gauge._h, float(kappa),
                                             int(nf), _ptr(uu), _dev(eta_global, "torch.complex128"),
                                             _dev(chi, "torch.complex128"), float(tol), int(maxit),
                                             ctypes.byref(params), _ptr(its), _ptr(rel), ctypes.byref(stats)),
                         allow=(DD_ENOCONV,))
        return chi, its, rel, self._wstats(stats), st

    def mb_log_reweight(self, blocks: Blocks, gauge: Gauge, domain: Blocks, domain_gauge: Gauge, kappa, N, c,
                        order, eta_global, params=None):
        """Stochastic estimate of ln W_N (eq. rw) with the caller's noise eta [n_vec, V, 4, 3]: (per-vector
        terms [n_vec] complex, their mean, info, status)."""
        nv = eta_global.shape[0]
        if params is None:
            params = solve_params(tol=1e-12)
        terms = np.zeros(2 * nv, dtype=np.float64)
        est = np.zeros(2, dtype=np.float64)
        stats = SolveStats(None, None, None, 0.0, 0, 0, 0, 0)
        st = self._check(_lib.dd_mb_log_reweight(self._h, blocks._h, gauge._h, domain._h, domain_gauge._h,
                                                 float(kappa), int(N), float(c), int(order), int(nv),
                                                 _dev(eta_global, "torch.complex128"), ctypes.byref(params),
                                                 _ptr(terms), _ptr(est), ctypes.byref(stats)),
                         allow=(DD_ENOCONV,))
        return terms[0::2] + 1j * terms[1::2], complex(est[0], est[1]), self._wstats(stats), st

    def mb_exterior_source(self, blocks: Blocks, gauge: Gauge, kappa, chi_global, xi, parts=3):
        """xi += the hops of chi_global [n_fields, V, 4, 3] from the sites of dPi outside each block's box
        into the box (parts 1: dPi_1, 2: dLambda_0, 3: both); xi [n_fields, total_sites, 4, 3]."""
        nf = chi_global.shape[0]
        self._check(_lib.dd_mb_exterior_source(self._h, blocks._h, gauge._h, float(kappa), int(nf),
                                               _dev(chi_global, "torch.complex128"), _dev(xi, "torch.complex128"),
                                               int(parts)))
        return xi

    # tuning
    def tune_set(self, what, value):
        """what: TUNE_RHS_GROUP_F64 / TUNE_RHS_GROUP_F32 (value 0 = auto, 1, 2 or 4), TUNE_HOP_LDS (0/1),
        TUNE_GMRES_THREADS (0, 256, 512), TUNE_GMRES_QUEUES (0, 1, 8), TUNE_GMRES_WG_PER_CU (0 = all that fit),
        TUNE_MB_FIELDS, TUNE_NN_KERNEL (0/1), TUNE_HOP_WALK (-1 off, 0 auto, n segments),
        TUNE_GMRES_REORTH (0 default, -1 never, 1..100 percent) or TUNE_BICG_FUSE (0 where possible,
        -1 never) or TUNE_DHAT_WALK (0 where possible, -1 never)."""
        self._check(_lib.dd_tune_set(self._h, int(what), int(value)))

    def autotune_bicgstab(self, blocks: Blocks, gauge: Gauge, kappa, b, params=None, cache=None, scratch=None):
        """Times the BiCGStab configurations on full solves of b and keeps the fastest (cache: a JSON file
        path; a stored entry for this problem is applied without timing).  Returns (list of (rhs_group,
        dhat_walk, dhat_rhs, bicg_fuse, ms), from_cache)."""
        import torch

        n_rhs = b.numel() // (blocks.total_sites * 12)
        if params is None:
            params = solve_params()
        x = scratch if scratch is not None else torch.empty_like(b)
        buf = (BicgTuneResult * 16)()
        n = _I32()
        hit = _I32()
        self._check(_lib.dd_autotune_bicgstab(self._h, blocks._h, gauge._h, float(kappa),
                                              _dev(b, "torch.complex128"), _dev(x, "torch.complex128"), int(n_rhs),
                                              ctypes.byref(params), cache.encode() if cache else None, buf, 16,
                                              ctypes.byref(n), ctypes.byref(hit)))
        out = [(r.rhs_group, r.dhat_walk, r.dhat_rhs, r.bicg_fuse, r.ms) for r in buf[:n.value]]
        return out, bool(hit.value)

    def autotune_gmres(self, blocks: Blocks, gauge: Gauge, kappa, b, params=None, scratch=None):
        """Times the persistent GMRES schedules on b's first inner solve and keeps the fastest.
        Returns (list of (threads, queues, wg_per_cu, ms), the chosen tuple)."""
        import torch

        n_rhs = b.numel() // (blocks.total_sites * 12)
        x = scratch if scratch is not None else torch.empty_like(b)
        if params is None:
            params = solve_params(method=GMRES)
        res = (TuneResult * 16)()
        n = _I32()
        self._check(_lib.dd_autotune_gmres(self._h, blocks._h, gauge._h, float(kappa), _dev(b, "torch.complex128"),
                                           _dev(x, "torch.complex128"), int(n_rhs), ctypes.byref(params), res, 16,
                                           ctypes.byref(n)))
        out = [(r.threads, r.queues, r.wg_per_cu, r.ms) for r in res[:min(n.value, 16)]]
        return out, min(out, key=lambda r: r[3])

    # learned preconditioner
    def nn_create(self, extent, weights, act=NN_LINEAR):
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32).reshape(-1))
        if w.size != nn_num_weights():
            raise ValueError("expected %d weights" % nn_num_weights())
        h = _P()
        self._check(_lib.dd_nn_create(self._h, _i32(extent).ctypes.data_as(_P), int(act),
                                      w.ctypes.data_as(_P), ctypes.byref(h)))
        return Net(h, self, tuple(int(v) for v in extent), act)

    # timing
    def timer_enable(self, on=True):
        self._check(_lib.dd_timer_enable(self._h, 1 if on else 0))

    def timer_reset(self):
        self._check(_lib.dd_timer_reset(self._h))

    def timer_read(self, kclass=KCLASS_HOP_F32):
        ms, n, b = _D(), _I64(), _D()
        self._check(_lib.dd_timer_read(self._h, int(kclass), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)))
        return ms.value, n.value, b.value
