"""ctypes binding of libhk (include/hk.h): the same entry points, argument marshalling only.

Every step of an iteration runs in libhk's HIP kernels. torch is used for device memory (state and
workspace buffers, uploaded inputs) and for the current stream. Importing this module fails loudly
when libhk.so has not been built.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhk.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "hk.h")

HK_OK = 0
HK_E_INVALID_ARG = -1
HK_E_BAD_STATE = -2
HK_E_SMALL_BUFFER = -3
HK_E_HIP = -4
HK_E_UNSUPPORTED = -5
HK_MODE_PPM = 0
HK_MODE_VCM = 1
HK_STATS_LUMA = 0
HK_STATS_RGB = 1

_fp = ctypes.POINTER(ctypes.c_float)
_vp = ctypes.c_void_p


class hk_params(ctypes.Structure):
    _fields_ = [
        ("r1", ctypes.c_float), ("k", ctypes.c_float), ("alpha_f", ctypes.c_double), ("alpha", ctypes.c_double),
        ("rmin", ctypes.c_double), ("n_a", ctypes.c_int32), ("n_s", ctypes.c_int32), ("mode", ctypes.c_int32),
        ("stats_channel", ctypes.c_int32), ("normal_cos_min", ctypes.c_float), ("max_iters", ctypes.c_int32),
        ("cell_scale", ctypes.c_float), ("cell_quantile", ctypes.c_float), ("heavy_cost", ctypes.c_int32),
        ("lanes_light", ctypes.c_int32), ("lanes_heavy", ctypes.c_int32), ("reserved", ctypes.c_int32 * 5),
    ]


class hk_photons(ctypes.Structure):
    _fields_ = [
        ("J_emitted", ctypes.c_uint64), ("n_stored", ctypes.c_int64),
        ("pos", _vp * 3), ("nrm", _vp * 3), ("flux", _vp * 3), ("mis", _vp * 3),
    ]


class hk_box_scene(ctypes.Structure):
    _fields_ = [("light", ctypes.c_float * 3), ("sphere_c", ctypes.c_float * 3), ("sphere_r", ctypes.c_float),
                ("power", ctypes.c_float)]


class HKError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libhk error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run `python paper_2504_04411_amd/build.py`")
        L = ctypes.CDLL(LIB_PATH)
        c = ctypes
        sig = {
            "hk_default_params": ([c.c_double, c.POINTER(hk_params)], c.c_int),
            "hk_create": ([c.POINTER(hk_params), c.POINTER(_vp)], c.c_int),
            "hk_destroy": ([_vp], c.c_int),
            "hk_state_bytes": ([_vp, c.c_int64, c.POINTER(c.c_size_t)], c.c_int),
            "hk_workspace_bytes": ([_vp, c.c_int64, c.c_int64, c.POINTER(c.c_size_t)], c.c_int),
            "hk_workspace_bytes_batch": ([_vp, c.c_int, c.POINTER(c.c_int64), c.POINTER(c.c_int64),
                                          c.POINTER(c.c_size_t)], c.c_int),
            "hk_get_params": ([_vp, c.POINTER(hk_params)], c.c_int),
            "hk_set_tuning": ([_vp, c.c_float, c.c_int, c.c_int, c.c_int], c.c_int),
            "hk_graph_create": ([_vp, c.c_int, c.POINTER(c.c_int), c.POINTER(hk_photons), c.POINTER(_vp), _vp,
                                 c.c_size_t, c.POINTER(_vp)], c.c_int),
            "hk_graph_create_box": ([_vp, c.c_int, c.POINTER(c.c_int), c.POINTER(hk_box_scene),
                                     c.POINTER(c.c_uint64), c.POINTER(hk_photons), c.POINTER(_vp), _vp, c.c_size_t,
                                     c.c_int, c.POINTER(_vp)], c.c_int),
            "hk_emit_box": ([_vp, c.c_int, _vp, c.POINTER(hk_box_scene), c.c_uint64, c.c_int64, _vp * 3, _vp * 3,
                             _vp * 3, _vp * 3, _vp], c.c_int),
            "hk_connect_box": ([_vp, c.c_int, _vp, c.POINTER(hk_box_scene), c.c_uint64, _vp], c.c_int),
            "hk_graph_launch": ([_vp, _vp], c.c_int),
            "hk_graph_destroy": ([_vp], c.c_int),
            "hk_autotune": ([_vp, c.c_int, c.POINTER(c.c_int), c.POINTER(hk_photons), c.POINTER(_vp),
                             c.POINTER(_vp), _vp, c.c_size_t, _vp, c.POINTER(hk_params)], c.c_int),
            "hk_set_kernels": ([_vp, c.c_int, c.c_int64, c.c_double, c.c_double, _vp * 3, c.c_void_p, _vp,
                                c.c_void_p, c.c_void_p, _vp, _vp, c.c_size_t, _vp], c.c_int),
            "hk_iterate": ([_vp, c.c_int, c.POINTER(c.c_int), c.POINTER(hk_photons), c.POINTER(_vp), _vp,
                            c.c_size_t, _vp], c.c_int),
            "hk_iterate_static": ([_vp, c.c_int, c.POINTER(c.c_int), c.POINTER(hk_photons), c.POINTER(_vp), _vp],
                                  c.c_int),
            "hk_read_radiance": ([_vp, c.c_int, _vp, _vp * 3, _vp], c.c_int),
            "hk_read_radii": ([_vp, c.c_int, _vp, _vp, _vp], c.c_int),
            "hk_read_debug": ([_vp, c.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp], c.c_int),
            "hk_read_sums": ([_vp, c.c_int, _vp, _vp, _vp, _vp, _vp], c.c_int),
            "hk_read_stats": ([_vp, c.c_int, _vp, _vp, _vp], c.c_int),
            "hk_f_quantile": ([c.c_double, c.c_double, c.c_double], c.c_double),
            "hk_profile_enable": ([_vp, c.c_int], c.c_int),
            "hk_profile_read": ([_vp, c.POINTER(c.c_double), c.c_int], c.c_int),
            "hk_gather_phases": ([_vp, c.c_int, c.POINTER(c.c_int), c.POINTER(hk_photons), c.POINTER(c.c_int)],
                                 c.c_int),
            "hk_mlp_param_count": ([], c.c_int),
            "hk_mlp_state_bytes": ([c.POINTER(c.c_size_t)], c.c_int),
            "hk_mlp_workspace_bytes": ([c.c_int64, c.POINTER(c.c_size_t)], c.c_int),
            "hk_mlp_set_params": ([_vp, _vp, _vp, _vp], c.c_int),
            "hk_mlp_get_params": ([_vp, _vp, _vp, _vp], c.c_int),
            "hk_mlp_forward": ([_vp, _vp, _vp, c.c_int64, _vp, _vp], c.c_int),
            "hk_mlp_grad": ([_vp, _vp, _vp, _vp, c.c_int64, _vp, _vp, c.c_size_t, _vp], c.c_int),
            "hk_mlp_train_step": ([_vp, _vp, _vp, _vp, c.c_int64, c.c_float, _vp, c.c_size_t, _vp], c.c_int),
            "hk_mlp_features": ([_vp, c.c_int, _vp, c.POINTER(hk_photons), c.c_float, _vp, _vp, _vp, c.c_size_t, _vp],
                                c.c_int),
            "hk_mlp_propose": ([_vp, c.c_int, _vp, _vp, c.c_float, _vp], c.c_int),
            "hk_version": ([], c.c_int),
            "hk_last_error": ([], c.c_char_p),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def header_functions():
    """Names of the functions declared in include/hk.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(hk_\w+)\s*\(", txt, flags=re.M)))


def check(rc: int):
    if rc != HK_OK:
        raise HKError(rc, lib().hk_last_error().decode())
    return rc


def _arr3(ptrs):
    a = (_vp * 3)()
    if ptrs is not None:
        for i, p in enumerate(ptrs):
            a[i] = p
    return a


def _opt3(ptrs):
    """Pointer to a 3-array of pointers, or NULL."""
    if ptrs is None:
        return None
    a = _arr3(ptrs)
    return ctypes.cast(a, ctypes.c_void_p), a


# ---------------------------------------------------------------------------------------------
# entry points with the header's names (plain integers for device pointers and streams)
# ---------------------------------------------------------------------------------------------

def hk_default_params(r1: float) -> hk_params:
    p = hk_params()
    check(lib().hk_default_params(float(r1), ctypes.byref(p)))
    return p


def hk_create(p: hk_params) -> int:
    h = _vp()
    check(lib().hk_create(ctypes.byref(p), ctypes.byref(h)))
    return h.value


def hk_destroy(ctx: int):
    check(lib().hk_destroy(ctx))


def hk_state_bytes(ctx: int, n: int) -> int:
    out = ctypes.c_size_t()
    check(lib().hk_state_bytes(ctx, int(n), ctypes.byref(out)))
    return out.value


def hk_workspace_bytes(ctx: int, max_photons: int, max_kernels: int) -> int:
    out = ctypes.c_size_t()
    check(lib().hk_workspace_bytes(ctx, int(max_photons), int(max_kernels), ctypes.byref(out)))
    return out.value


def hk_workspace_bytes_batch(ctx: int, n_photons, n_kernels) -> int:
    n = len(n_photons)
    out = ctypes.c_size_t()
    a = (ctypes.c_int64 * n)(*[int(x) for x in n_photons])
    b = (ctypes.c_int64 * n)(*[int(x) for x in n_kernels])
    check(lib().hk_workspace_bytes_batch(ctx, n, a, b, ctypes.byref(out)))
    return out.value


def hk_get_params(ctx: int) -> hk_params:
    p = hk_params()
    check(lib().hk_get_params(ctx, ctypes.byref(p)))
    return p


def hk_set_tuning(ctx: int, cell_scale: float, heavy_cost: int, lanes_light: int, lanes_heavy: int):
    check(lib().hk_set_tuning(ctx, float(cell_scale), int(heavy_cost), int(lanes_light), int(lanes_heavy)))


def hk_set_kernels(ctx, set_id, n, r1, rmin, pos, nrm, r_init, cam_beta, cam_mis, state, workspace, workspace_bytes,
                   stream):
    keep = []
    args = []
    for x in (nrm, cam_beta, cam_mis):
        o = _opt3(x)
        if o is None:
            args.append(None)
        else:
            args.append(o[0])
            keep.append(o[1])
    check(lib().hk_set_kernels(ctx, int(set_id), int(n), float(r1), float(rmin), _arr3(pos), args[0], r_init,
                               args[1], args[2], state, workspace, int(workspace_bytes), stream))


def make_photons(J_emitted, n_stored, pos, flux, nrm=None, mis=None) -> hk_photons:
    ph = hk_photons()
    ph.J_emitted = int(J_emitted)
    ph.n_stored = int(n_stored)
    ph.pos = _arr3(pos)
    ph.flux = _arr3(flux)
    ph.nrm = _arr3(nrm)
    ph.mis = _arr3(mis)
    return ph


def hk_iterate(ctx, set_ids, photons, states, workspace, workspace_bytes, stream):
    n = len(set_ids)
    ids = (ctypes.c_int * n)(*set_ids)
    phs = (hk_photons * n)(*photons)
    sts = (_vp * n)(*states)
    check(lib().hk_iterate(ctx, n, ids, phs, sts, workspace, int(workspace_bytes), stream))


def hk_iterate_static(ctx, set_ids, photons, states, stream):
    n = len(set_ids)
    ids = (ctypes.c_int * n)(*set_ids)
    phs = (hk_photons * n)(*photons)
    sts = (_vp * n)(*states)
    check(lib().hk_iterate_static(ctx, n, ids, phs, sts, stream))


HK_STATIC_SCRATCH_BYTES = 64 << 20


def _set_arrays(set_ids, photons, states):
    n = len(set_ids)
    return (n, (ctypes.c_int * n)(*set_ids), (hk_photons * n)(*photons), (_vp * n)(*states))


def hk_graph_create(ctx, set_ids, photons, states, workspace, workspace_bytes) -> int:
    n, ids, phs, sts = _set_arrays(set_ids, photons, states)
    g = _vp()
    check(lib().hk_graph_create(ctx, n, ids, phs, sts, workspace, int(workspace_bytes), ctypes.byref(g)))
    return g.value


def box_scene(light, sphere_c, sphere_r, power) -> hk_box_scene:
    sc = hk_box_scene()
    sc.light[:] = [float(v) for v in light]
    sc.sphere_c[:] = [float(v) for v in sphere_c]
    sc.sphere_r = float(sphere_r)
    sc.power = float(power)
    return sc


HK_BOX_CONNECT = 1


def hk_emit_box(ctx, set_id, state, scene: hk_box_scene, seed, J, pos, nrm, flux, stream, mis=None):
    check(lib().hk_emit_box(ctx, int(set_id), state, ctypes.byref(scene), int(seed), int(J), _arr3(pos), _arr3(nrm),
                            _arr3(flux), _arr3(mis), stream))


def hk_connect_box(ctx, set_id, state, scene: hk_box_scene, J_emitted, stream):
    check(lib().hk_connect_box(ctx, int(set_id), state, ctypes.byref(scene), int(J_emitted), stream))


def hk_graph_create_box(ctx, set_ids, scenes, seeds, photons, states, workspace, workspace_bytes, flags=0) -> int:
    n, ids, phs, sts = _set_arrays(set_ids, photons, states)
    scs = (hk_box_scene * n)(*scenes)
    sds = (ctypes.c_uint64 * n)(*[int(x) for x in seeds])
    g = _vp()
    check(lib().hk_graph_create_box(ctx, n, ids, scs, sds, phs, sts, workspace, int(workspace_bytes), int(flags),
                                    ctypes.byref(g)))
    return g.value


def hk_graph_launch(graph, stream):
    check(lib().hk_graph_launch(graph, stream))


def hk_graph_destroy(graph):
    check(lib().hk_graph_destroy(graph))


def hk_autotune(ctx, set_ids, photons, states, scratch, workspace, workspace_bytes, stream) -> hk_params:
    n, ids, phs, sts = _set_arrays(set_ids, photons, states)
    scr = (_vp * n)(*scratch)
    p = hk_params()
    check(lib().hk_autotune(ctx, n, ids, phs, sts, scr, workspace, int(workspace_bytes), stream, ctypes.byref(p)))
    return p


def hk_read_radiance(ctx, set_id, state, out_rgb, stream):
    check(lib().hk_read_radiance(ctx, int(set_id), state, _arr3(out_rgb), stream))


def hk_read_radii(ctx, set_id, state, out, stream):
    check(lib().hk_read_radii(ctx, int(set_id), state, out, stream))


def hk_read_debug(ctx, set_id, state, count, F, Fc, decision, t, stream):
    check(lib().hk_read_debug(ctx, int(set_id), state, count, F, Fc, decision, t, stream))


def hk_read_sums(ctx, set_id, state, S, Q, tau, stream):
    check(lib().hk_read_sums(ctx, int(set_id), state, S, Q, tau, stream))


def hk_read_stats(ctx, set_id, state, out, stream):
    check(lib().hk_read_stats(ctx, int(set_id), state, out, stream))


def hk_f_quantile(d1: float, d2: float, alpha: float) -> float:
    return lib().hk_f_quantile(float(d1), float(d2), float(alpha))


def hk_profile_enable(ctx, on: bool):
    check(lib().hk_profile_enable(ctx, 1 if on else 0))


def hk_profile_read(ctx):
    out = (ctypes.c_double * 10)()
    check(lib().hk_profile_read(ctx, out, 10))
    return list(out)


def hk_gather_phases(ctx, set_ids, photons):
    n = len(set_ids)
    ids = (ctypes.c_int * n)(*set_ids)
    phs = (hk_photons * n)(*photons)
    out = (ctypes.c_int * n)()
    check(lib().hk_gather_phases(ctx, n, ids, phs, out))
    return list(out)


def hk_mlp_param_count() -> int:
    return lib().hk_mlp_param_count()


def hk_mlp_state_bytes() -> int:
    out = ctypes.c_size_t()
    check(lib().hk_mlp_state_bytes(ctypes.byref(out)))
    return out.value


def hk_mlp_workspace_bytes(n: int) -> int:
    out = ctypes.c_size_t()
    check(lib().hk_mlp_workspace_bytes(int(n), ctypes.byref(out)))
    return out.value


def hk_mlp_set_params(ctx, mlp, theta, stream):
    check(lib().hk_mlp_set_params(ctx, mlp, theta, stream))


def hk_mlp_get_params(ctx, mlp, theta_out, stream):
    check(lib().hk_mlp_get_params(ctx, mlp, theta_out, stream))


def hk_mlp_forward(ctx, mlp, feat, n, y, stream):
    check(lib().hk_mlp_forward(ctx, mlp, feat, int(n), y, stream))


def hk_mlp_grad(ctx, mlp, feat, label, n, grad_out, ws, ws_bytes, stream):
    check(lib().hk_mlp_grad(ctx, mlp, feat, label, int(n), grad_out, ws, int(ws_bytes), stream))


def hk_mlp_train_step(ctx, mlp, feat, label, n, lr, ws, ws_bytes, stream):
    check(lib().hk_mlp_train_step(ctx, mlp, feat, label, int(n), float(lr), ws, int(ws_bytes), stream))


def hk_mlp_features(ctx, set_id, state, photons, it_code, feat, counts, ws, ws_bytes, stream):
    check(lib().hk_mlp_features(ctx, int(set_id), state, ctypes.byref(photons), float(it_code), feat, counts, ws,
                                int(ws_bytes), stream))


def hk_mlp_propose(ctx, set_id, state, y, margin, stream):
    check(lib().hk_mlp_propose(ctx, int(set_id), state, y, float(margin), stream))


def hk_version() -> int:
    return lib().hk_version()


def hk_last_error() -> str:
    return lib().hk_last_error().decode()
