"""ctypes binding of ``libtuckfmm.so``: the C ABI of ``include/tuckfmm.h``, one Python
function per C entry point with the same name.  Argument marshalling only: every
computation runs in the library's HIP kernels.

Device buffers are torch tensors on the current HIP device (``data_ptr()`` is
passed); host buffers are NumPy arrays.  ``stream=None`` means torch's current
stream.  A non-OK status raises :class:`FmmError` carrying the library's message.
If the shared library has not been built, importing this module raises
``ImportError``: there is no fallback path.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtuckfmm.so")

__all__ = [
    "FMM_OK", "FMM_C128", "FMM_C64", "FMM_BF16X2", "FMM_BF16X3", "FmmError", "Layout", "exported_symbols",
    "fmm_last_error", "fmm_version", "fmm_device_count",
    "fmm_geometry_build", "fmm_geometry_info", "fmm_geometry_tables", "fmm_geometry_layout", "fmm_geometry_boxes",
    "fmm_farfield_fill", "fmm_planewave_excitation",
    "fmm_geometry_destroy", "fmm_tucker_create", "fmm_farfield_compress", "fmm_farfield_compress_svd",
    "fmm_tucker_set_group", "fmm_tucker_set_box_grid", "fmm_tucker_save", "fmm_tucker_load",
    "fmm_tucker_layout",
    "fmm_tucker_ranks", "fmm_tucker_export", "fmm_tucker_storage_bytes", "fmm_tucker_upload",
    "fmm_tucker_aggregate", "fmm_tucker_disaggregate", "fmm_tucker_pass", "fmm_tucker_pass_noalloc",
    "fmm_graph_capture", "fmm_graph_launch",
    "fmm_tucker_tune", "fmm_tucker_set_tuned", "fmm_tucker_destroy", "fmm_dense_create", "fmm_dense_aggregate",
    "fmm_dense_disaggregate",
    "fmm_dense_destroy",
]

FMM_OK = 0
STATUS = {0: "FMM_OK", -1: "FMM_ERR_ARG", -2: "FMM_ERR_SHAPE", -3: "FMM_ERR_SIZE", -4: "FMM_ERR_DEVICE",
          -5: "FMM_ERR_NUMERIC", -6: "FMM_ERR_UNSUPPORTED", -7: "FMM_ERR_STATE",
          -8: "FMM_ERR_IO"}
FMM_C128, FMM_C64, FMM_BF16X2, FMM_BF16X3 = 0, 1, 2, 3

if not os.path.exists(LIB_PATH):
    raise ImportError("libtuckfmm.so is not built; run `python paper_2103_05822_amd/build.py` "
                      "or __graft_entry__.build() first")
# torch brings its own HIP runtime (SONAME libamdhip64.so.7).  Loading torch first makes
# the library's libamdhip64.so.7 / librocblas.so.5 dependencies resolve to the copies
# torch already mapped, so the process has one HIP runtime and the library can use
# torch's allocations and streams.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)


class FmmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status


class fmm_layout(ctypes.Structure):
    _fields_ = [("n_theta", ctypes.c_int32), ("n_phi", ctypes.c_int32), ("n_groups", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("offsets", ctypes.POINTER(ctypes.c_int64))]


class fmm_tune_result(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("tile_steps", ctypes.c_int32), ("rhs_chunk", ctypes.c_int32),
                ("threads", ctypes.c_int32), ("ms", ctypes.c_float), ("order", ctypes.c_int32),
                ("from_cache", ctypes.c_int32)]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_f64 = ctypes.c_double
_sz = ctypes.c_size_t
_st = ctypes.c_int

_SIGS = {
    "fmm_last_error": (ctypes.c_char_p, []),
    "fmm_version": (ctypes.c_char_p, []),
    "fmm_device_count": (_i32, []),
    "fmm_geometry_build": (_st, [_vp, _i64, _vp, _i64, _vp, _f64, _i32, _f64, _i32, _i32, ctypes.POINTER(_vp)]),
    "fmm_geometry_info": (_st, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i32)]),
    "fmm_geometry_tables": (_st, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "fmm_geometry_layout": (_st, [_vp, ctypes.POINTER(fmm_layout)]),
    "fmm_geometry_boxes": (_st, [_vp, _vp, _vp]),
    "fmm_farfield_fill": (_st, [_vp, _i32, _i32, _vp, _vp]),
    "fmm_planewave_excitation": (_st, [_vp, _i32, _vp, _vp, _st, _vp, _vp]),
    "fmm_geometry_destroy": (None, [_vp]),
    "fmm_tucker_create": (_st, [ctypes.POINTER(fmm_layout), ctypes.POINTER(_vp)]),
    "fmm_farfield_compress": (_st, [ctypes.POINTER(fmm_layout), _vp, _i32, _i32, _f64, _vp, ctypes.POINTER(_vp)]),
    "fmm_farfield_compress_svd": (_st, [ctypes.POINTER(fmm_layout), _vp, _i32, _i32, _f64, _vp,
                                        ctypes.POINTER(_vp)]),
    "fmm_tucker_set_group": (_st, [_vp, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp]),
    "fmm_tucker_set_box_grid": (_st, [_vp, _i32, _i32, _i32, _vp]),
    "fmm_tucker_save": (_st, [_vp, ctypes.c_char_p]),
    "fmm_tucker_layout": (_st, [_vp, ctypes.POINTER(fmm_layout)]),
    "fmm_tucker_load": (_st, [ctypes.c_char_p, ctypes.POINTER(_vp)]),
    "fmm_tucker_ranks": (_st, [_vp, _vp]),
    "fmm_tucker_export": (_st, [_vp, _i32, _i32, _st, _vp, _vp, _vp, _vp]),
    "fmm_tucker_storage_bytes": (_st, [_vp, _st, ctypes.POINTER(_sz), ctypes.POINTER(_sz)]),
    "fmm_tucker_upload": (_st, [_vp, _st, _vp, _sz, _vp]),
    "fmm_tucker_aggregate": (_st, [_vp, _st, _i32, _vp, _vp, _vp]),
    "fmm_tucker_disaggregate": (_st, [_vp, _st, _i32, _vp, _vp, _vp]),
    "fmm_tucker_pass": (_st, [_vp, _st, _i32, _vp, _vp, _vp, _vp, _vp]),
    "fmm_tucker_pass_noalloc": (_st, [_vp, _st, _i32, _vp, _vp, _vp, _vp, _vp]),
    "fmm_graph_capture": (_st, [_vp, _st, _i32, _vp, _vp, _vp, _vp, _vp]),
    "fmm_graph_launch": (_st, [_vp, _vp]),
    "fmm_tucker_tune": (_st, [_vp, _st, _i32, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(fmm_tune_result)]),
    "fmm_tucker_set_tuned": (_st, [_vp, _st, _i32, ctypes.POINTER(fmm_tune_result)]),
    "fmm_tucker_destroy": (None, [_vp]),
    "fmm_dense_create": (_st, [ctypes.POINTER(fmm_layout), ctypes.POINTER(_vp)]),
    "fmm_dense_aggregate": (_st, [_vp, _st, _vp, _i32, _vp, _vp, _vp]),
    "fmm_dense_disaggregate": (_st, [_vp, _st, _vp, _i32, _vp, _vp, _vp]),
    "fmm_dense_destroy": (None, [_vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def exported_symbols():
    """Names of the C entry points this binding declares."""
    return sorted(_SIGS)


def _check(status):
    if status != FMM_OK:
        raise FmmError(status, _lib.fmm_last_error().decode())
    return status


def _ptr(t):
    """Device or host address of a torch tensor / NumPy array (None -> NULL)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        if not torch.cuda.is_available():
            return None          # the library reports FMM_ERR_DEVICE itself
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _c128(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


# ----------------------------------------------------------------------- misc

def fmm_last_error():
    return _lib.fmm_last_error().decode()


def fmm_version():
    return _lib.fmm_version().decode()


def fmm_device_count():
    return int(_lib.fmm_device_count())


# ------------------------------------------------------------------- geometry

class Layout:
    """Owns the offsets array behind an ``fmm_layout``."""

    def __init__(self, n_theta, n_phi, offsets):
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        self.n_theta, self.n_phi = int(n_theta), int(n_phi)
        self.n_groups = self.offsets.size - 1
        self.c = fmm_layout(self.n_theta, self.n_phi, self.n_groups, 0,
                            self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))

    @property
    def n_basis(self):
        return int(self.offsets[-1])

    @property
    def n_dir(self):
        return self.n_theta * self.n_phi


def fmm_geometry_build(verts, tris, origin, box, boxes_per_axis, wavenumber, n_theta, n_phi):
    v = np.ascontiguousarray(verts, dtype=np.float64)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    o = np.ascontiguousarray(origin, dtype=np.float64)
    out = _vp()
    _check(_lib.fmm_geometry_build(v.ctypes.data, v.shape[0], t.ctypes.data, t.shape[0], o.ctypes.data,
                                   float(box), int(boxes_per_axis), float(wavenumber), int(n_theta),
                                   int(n_phi), ctypes.byref(out)))
    return out.value


def fmm_geometry_info(geom):
    n, g = _i64(), _i32()
    _check(_lib.fmm_geometry_info(geom, ctypes.byref(n), ctypes.byref(g)))
    return int(n.value), int(g.value)


def fmm_geometry_tables(geom):
    n, g = fmm_geometry_info(geom)
    lay = fmm_layout()
    _check(_lib.fmm_geometry_layout(geom, ctypes.byref(lay)))
    offsets = np.empty(g + 1, np.int64)
    perm = np.empty(n, np.int64)
    centers = np.empty((g, 3), np.float64)
    theta = np.empty(lay.n_theta, np.float64)
    phi = np.empty(lay.n_phi, np.float64)
    _check(_lib.fmm_geometry_tables(geom, offsets.ctypes.data, perm.ctypes.data, centers.ctypes.data,
                                    theta.ctypes.data, phi.ctypes.data))
    return {"offsets": offsets, "perm": perm, "centers": centers, "theta": theta, "phi": phi}


def fmm_geometry_layout(geom):
    lay = fmm_layout()
    _check(_lib.fmm_geometry_layout(geom, ctypes.byref(lay)))
    tabs = fmm_geometry_tables(geom)
    return Layout(lay.n_theta, lay.n_phi, tabs["offsets"])


def fmm_geometry_boxes(geom):
    """(K, box_of_group int64 [n_groups]): the K x K x K box grid and each group's box."""
    _, g = fmm_geometry_info(geom)
    k = _i32()
    boxes = np.empty(g, np.int64)
    _check(_lib.fmm_geometry_boxes(geom, ctypes.byref(k), boxes.ctypes.data))
    return int(k.value), boxes


def fmm_farfield_fill(geom, first_group, count, farfield, stream=None):
    _check(_lib.fmm_farfield_fill(geom, int(first_group), int(count), _ptr(farfield), _stream(stream)))


def fmm_planewave_excitation(geom, khat, epol, prec, x, stream=None):
    """Excitation vectors of the plane waves (khat, epol: [nrhs, 3] float64 host arrays)
    into the device tensor x [N, nrhs] (complex128 for FMM_C128, else complex64)."""
    khat = np.ascontiguousarray(np.atleast_2d(khat), dtype=np.float64)
    epol = np.ascontiguousarray(np.atleast_2d(epol), dtype=np.float64)
    if khat.shape != epol.shape or khat.shape[1] != 3:
        raise ValueError("khat and epol must both be [nrhs, 3]")
    _check(_lib.fmm_planewave_excitation(geom, int(khat.shape[0]), khat.ctypes.data, epol.ctypes.data, int(prec),
                                         _ptr(x), _stream(stream)))


def fmm_geometry_destroy(geom):
    _lib.fmm_geometry_destroy(geom)


# --------------------------------------------------------------------- Tucker

def fmm_tucker_create(layout):
    out = _vp()
    _check(_lib.fmm_tucker_create(ctypes.byref(layout.c), ctypes.byref(out)))
    return out.value


def fmm_farfield_compress(layout, farfield, first_group, count, gamma, handle=None, stream=None):
    h = _vp(handle)
    _check(_lib.fmm_farfield_compress(ctypes.byref(layout.c), _ptr(farfield), int(first_group), int(count),
                                      float(gamma), _stream(stream), ctypes.byref(h)))
    return h.value


def fmm_farfield_compress_svd(layout, farfield, first_group, count, gamma, handle=None, stream=None):
    h = _vp(handle)
    _check(_lib.fmm_farfield_compress_svd(ctypes.byref(layout.c), _ptr(farfield), int(first_group), int(count),
                                          float(gamma), _stream(stream), ctypes.byref(h)))
    return h.value


def fmm_tucker_set_group(h, group, alpha, core, u_theta, u_phi, u_beta):
    core, ut, up, ub = (_c128(a) for a in (core, u_theta, u_phi, u_beta))
    rt, rp, rb = core.shape
    _check(_lib.fmm_tucker_set_group(h, int(group), int(alpha), rt, rp, rb, core.ctypes.data, ut.ctypes.data,
                                     up.ctypes.data, ub.ctypes.data))


def fmm_tucker_set_box_grid(h, dims, box_of_group):
    """dims = (K_x, K_y, K_z) and box_of_group [n_groups]; dims = None clears the grid."""
    if dims is None:
        _check(_lib.fmm_tucker_set_box_grid(h, 0, 0, 0, None))
        return
    boxes = np.ascontiguousarray(box_of_group, dtype=np.int64)
    kx, ky, kz = (int(d) for d in dims)
    _check(_lib.fmm_tucker_set_box_grid(h, kx, ky, kz, boxes.ctypes.data))


def fmm_tucker_save(h, path):
    _check(_lib.fmm_tucker_save(h, os.fsencode(path)))


def fmm_tucker_load(path):
    out = _vp()
    _check(_lib.fmm_tucker_load(os.fsencode(path), ctypes.byref(out)))
    return out.value


def fmm_tucker_layout(h):
    lay = fmm_layout()
    _check(_lib.fmm_tucker_layout(h, ctypes.byref(lay)))
    offsets = np.ctypeslib.as_array(lay.offsets, shape=(lay.n_groups + 1,)).copy()
    return Layout(lay.n_theta, lay.n_phi, offsets)


def fmm_tucker_ranks(h, n_groups):
    r = np.empty((n_groups, 2, 3), np.int32)
    _check(_lib.fmm_tucker_ranks(h, r.ctypes.data))
    return r


def fmm_tucker_export(h, group, alpha, ranks, n_theta, n_phi, n_beta, as_stored=FMM_C128):
    """Factors (core, U^theta, U^phi, U^beta) of one tensor as complex128 arrays;
    ``as_stored`` = the precision whose stored values to return (FMM_C128: FP64)."""
    rt, rp, rb = (int(v) for v in ranks)
    core = np.empty((rt, rp, rb), np.complex128)
    ut = np.empty((n_theta, rt), np.complex128)
    up = np.empty((n_phi, rp), np.complex128)
    ub = np.empty((n_beta, rb), np.complex128)
    _check(_lib.fmm_tucker_export(h, int(group), int(alpha), int(as_stored), core.ctypes.data, ut.ctypes.data,
                                  up.ctypes.data, ub.ctypes.data))
    return core, ut, up, ub


def fmm_tucker_storage_bytes(h, prec):
    fb, ab = _sz(), _sz()
    _check(_lib.fmm_tucker_storage_bytes(h, int(prec), ctypes.byref(fb), ctypes.byref(ab)))
    return int(fb.value), int(ab.value)


def fmm_tucker_upload(h, prec, arena, nbytes=None, stream=None):
    if nbytes is None:
        nbytes = arena.numel() * arena.element_size()
    _check(_lib.fmm_tucker_upload(h, int(prec), _ptr(arena), int(nbytes), _stream(stream)))


def fmm_tucker_aggregate(h, prec, nrhs, x, F, stream=None):
    _check(_lib.fmm_tucker_aggregate(h, int(prec), int(nrhs), _ptr(x), _ptr(F), _stream(stream)))


def fmm_tucker_disaggregate(h, prec, nrhs, G, V, stream=None):
    _check(_lib.fmm_tucker_disaggregate(h, int(prec), int(nrhs), _ptr(G), _ptr(V), _stream(stream)))


def fmm_tucker_pass(h, prec, nrhs, x, F, G, V, stream=None):
    _check(_lib.fmm_tucker_pass(h, int(prec), int(nrhs), _ptr(x), _ptr(F), _ptr(G), _ptr(V), _stream(stream)))


def fmm_tucker_pass_noalloc(h, prec, nrhs, x, F, G, V, stream=None):
    _check(_lib.fmm_tucker_pass_noalloc(h, int(prec), int(nrhs), _ptr(x), _ptr(F), _ptr(G), _ptr(V),
                                        _stream(stream)))


def fmm_graph_capture(h, prec, nrhs, x, F, G, V, stream):
    _check(_lib.fmm_graph_capture(h, int(prec), int(nrhs), _ptr(x), _ptr(F), _ptr(G), _ptr(V), _stream(stream)))


def fmm_graph_launch(h, stream=None):
    _check(_lib.fmm_graph_launch(h, _stream(stream)))


def fmm_tucker_tune(h, prec, nrhs, x, F, G, V, stream=None):
    """Returns a dict with the chosen path, tile_steps, rhs_chunk, threads, order, ms per
    pass and from_cache."""
    r = fmm_tune_result()
    _check(_lib.fmm_tucker_tune(h, int(prec), int(nrhs), _ptr(x), _ptr(F), _ptr(G), _ptr(V), _stream(stream),
                                ctypes.byref(r)))
    return {"path": r.path, "tile_steps": r.tile_steps, "rhs_chunk": r.rhs_chunk, "threads": r.threads,
            "order": r.order, "ms": r.ms, "from_cache": r.from_cache}


def fmm_tucker_set_tuned(h, prec, nrhs, path, tile_steps=0, rhs_chunk=0, threads=0, order=0):
    r = fmm_tune_result(int(path), int(tile_steps), int(rhs_chunk), int(threads), 0.0, int(order), 0)
    _check(_lib.fmm_tucker_set_tuned(h, int(prec), int(nrhs), ctypes.byref(r)))


def fmm_tucker_destroy(h):
    _lib.fmm_tucker_destroy(h)


# ---------------------------------------------------------------------- dense

def fmm_dense_create(layout):
    out = _vp()
    _check(_lib.fmm_dense_create(ctypes.byref(layout.c), ctypes.byref(out)))
    return out.value


def fmm_dense_aggregate(d, prec, farfield, nrhs, x, F, stream=None):
    _check(_lib.fmm_dense_aggregate(d, int(prec), _ptr(farfield), int(nrhs), _ptr(x), _ptr(F), _stream(stream)))


def fmm_dense_disaggregate(d, prec, farfield, nrhs, G, V, stream=None):
    _check(_lib.fmm_dense_disaggregate(d, int(prec), _ptr(farfield), int(nrhs), _ptr(G), _ptr(V),
                                       _stream(stream)))


def fmm_dense_destroy(d):
    _lib.fmm_dense_destroy(d)
