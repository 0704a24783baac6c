"""ctypes binding of libshamr (include/shamr.h): argument marshalling only.

Every step of the path runs in the HIP library; PyTorch supplies device memory (one
arena tensor per level) and the stream.  If the library is not built this module
raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, Structure, c_char_p, c_double, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libshamr.so")

SH_OK, SH_EINVAL, SH_ENOMEM, SH_ENEST, SH_ESTATE, SH_EDEVICE = range(6)
SH_F64, SH_F32 = 0, 1
ROLE_UN, ROLE_A, ROLE_B, ROLE_OLD = 0, 1, 2, 3
_STATUS = {1: "SH_EINVAL", 2: "SH_ENOMEM", 3: "SH_ENEST", 4: "SH_ESTATE", 5: "SH_EDEVICE"}


class ShError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class sh_params(Structure):
    _fields_ = [
        ("n0", c_int32), ("L", c_double), ("cfl", c_double), ("eta0", c_double),
        ("lam", c_double), ("alpha_fric", c_double), ("beta_pot", c_int32),
        ("max_level", c_int32), ("blocking_factor", c_int32), ("max_box", c_int32),
        ("n_error_buf", c_int32), ("prec", c_int32), ("integrator", c_int32), ("lap_order", c_int32),
        ("interp", c_int32), ("ko_order", c_int32), ("ko_eps", c_double), ("tee_fields", c_int32),
    ]


_PROTOS = {
    "sh_arena_bytes": (c_size_t, [POINTER(sh_params), c_int32, c_int32, POINTER(c_int32)]),
    "sh_hierarchy_create": (c_int32, [POINTER(sh_params), c_void_p, POINTER(c_void_p)]),
    "sh_set_level_layout": (c_int32, [c_void_p, c_int32, c_int32, POINTER(c_int32), c_void_p, c_size_t]),
    "sh_write_state": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_int32, c_int32]),
    "sh_read_state": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_int32, c_int32]),
    "sh_fill_ghosts": (c_int32, [c_void_p, c_int32, c_int32, c_int32]),
    "sh_advance_level": (c_int32, [c_void_p, c_int32, c_int32]),
    "sh_average_down": (c_int32, [c_void_p, c_int32]),
    "sh_tag_cells": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int64, POINTER(c_int64)]),
    "sh_tag_cells_noalloc": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int64, POINTER(c_int64)]),
    "sh_energy": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_int64)]),
    "sh_eval_rhs": (c_int32, [c_void_p, c_int32, c_void_p]),
    "sh_level_info": (c_int32, [c_void_p, c_int32, POINTER(c_int64), POINTER(c_double), POINTER(c_int32),
                                POINTER(c_int64)]),
    "sh_num_levels": (c_int32, [c_void_p]),
    "sh_cluster_tags": (c_int32, [c_void_p, c_int32, c_int64, c_void_p, c_double, c_void_p, c_int32,
                                  POINTER(c_int32)]),
    "sh_cluster_boxes": (c_int32, [c_int32, c_int32, c_void_p, c_int32, c_int32, c_int32, c_double, c_int64,
                                   c_void_p, c_void_p, c_int32, POINTER(c_int32)]),
    "sh_cluster_tags_carried": (c_int32, [c_void_p, c_int32, c_int64, c_void_p, c_int64, c_void_p, c_int32,
                                          c_double, c_void_p, c_int32, POINTER(c_int32)]),
    "sh_cluster_boxes_carried": (c_int32, [c_int32, c_int32, c_void_p, c_int32, c_int32, c_int32, c_double,
                                           c_int64, c_void_p, c_int64, c_void_p, c_int32, c_void_p, c_int32,
                                           POINTER(c_int32)]),
    "sh_tag_blocks": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_int64, POINTER(c_int64)]),
    "sh_cluster_blocks": (c_int32, [c_void_p, c_int32, c_void_p, c_int64, c_double, c_void_p, c_int32,
                                    POINTER(c_int32)]),
    "sh_cluster_boxes_bits": (c_int32, [c_int32, c_int32, c_void_p, c_int32, c_int32, c_double, c_void_p, c_int64,
                                        c_void_p, c_int32, POINTER(c_int32)]),
    "sh_dilate_octants": (c_int32, [c_int32, c_int32, c_void_p, c_void_p, c_int64]),
    "sh_local_tag_boxes": (c_int32, [c_int32, c_int32, c_void_p, c_int32, c_int32, c_int32, c_int64, c_void_p,
                                     c_void_p, c_int32, POINTER(c_int32)]),
    "sh_local_nest_boxes": (c_int32, [c_int32, c_int32, c_void_p, c_int32, c_void_p, c_int32, c_int32, c_void_p,
                                      c_int32, POINTER(c_int32)]),
    "sh_sync": (c_int32, [c_void_p]),
    "sh_hierarchy_destroy": (c_int32, [c_void_p]),
    "sh_last_error": (c_char_p, []),
    "sh_debug_stage_scalars": (c_int32, [c_void_p, c_int32, c_int32, POINTER(c_double)]),
    "sh_set_tuning": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_int32, c_int32, c_int32, c_int32]),
    "sh_profile": (c_int32, [c_void_p, c_int32]),
    "sh_profile_read": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_int64)]),
    "sh_batch_create": (c_int32, [c_int32, POINTER(c_void_p), POINTER(c_void_p)]),
    "sh_batch_advance": (c_int32, [c_void_p]),
    "sh_batch_destroy": (c_int32, [c_void_p]),
    "sh_trace": (c_int32, [c_void_p, c_int32]),
    "sh_trace_read": (c_int64, [c_void_p, c_void_p, c_int64]),
    "sh_capture_begin": (c_int32, [c_void_p]),
    "sh_capture_end": (c_int32, [c_void_p, POINTER(c_void_p)]),
    "sh_batch_capture": (c_int32, [c_void_p, c_int32, POINTER(c_void_p)]),
    "sh_graph_launch": (c_int32, [c_void_p]),
    "sh_graph_destroy": (c_int32, [c_void_p]),
    "sh_set_tee": (c_int32, [c_void_p, c_int32, c_double, c_int32]),
    "sh_shadow_begin": (c_int32, [c_void_p]),
    "sh_shadow_advance": (c_int32, [c_void_p]),
    "sh_shadow_end": (c_int32, [c_void_p]),
    "sh_read_tee": (c_int32, [c_void_p, c_int32, c_void_p]),
    "sh_set_tee_fields": (c_int32, [c_void_p, c_int32, POINTER(c_double), POINTER(c_double), c_int32]),
    "sh_field_absmax": (c_int32, [c_void_p, POINTER(c_double)]),
    "sh_stream_probe": (c_int32, [c_int32, c_void_p, c_void_p, c_int64, c_void_p]),
    "sh_set_debug": (c_int32, [c_void_p, c_int32]),
    "sh_set_stream": (c_int32, [c_void_p, c_void_p]),
    "sh_restart": (c_int32, [c_void_p]),
    "sh_batch_update": (c_int32, [c_void_p, c_int32, POINTER(c_void_p)]),
}

EXPORTED = tuple(_PROTOS)
_lib = None


def load(path: str = None):
    """Load libshamr.so (raises if it has not been built).  SHAMR_LIB in the environment
    names another build of the same library (the host-sanitizer build)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("SHAMR_LIB") or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it first (python -m paper_2404_02950_amd.build_lib)")
    # torch first: the library then binds to the HIP runtime torch has loaded (same soname)
    # instead of loading the system copy beside it, which would leave two HIP runtimes,
    # each with its own view of the device, in one process
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in _PROTOS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != SH_OK:
        raise ShError(status, _lib.sh_last_error().decode())


def _boxes_arr(boxes):
    b = np.ascontiguousarray(np.asarray(boxes, dtype=np.int32).reshape(-1, 6))
    return b, b.ctypes.data_as(POINTER(c_int32))


def box_shape(b):
    """(nz, ny, nx) of a box (x_lo, y_lo, z_lo, x_hi, y_hi, z_hi)."""
    return (b[5] - b[2] + 1, b[4] - b[1] + 1, b[3] - b[0] + 1)


def cluster_boxes(M: int, level_boxes, tags, blocking_factor: int = 8, max_box: int = 64,
                  n_error_buf: int = 2, efficiency: float = 0.7, carried=None, grow: int = 1):
    """Berger-Rigoutsos clustering of level tags into next-level boxes (host only).
    ``carried``: tags of the next finer level (its index space) clustered through their
    coarse parents grown by ``grow`` + n_error_buf cells (sh_cluster_boxes_carried)."""
    lib = load()
    lb = np.ascontiguousarray(np.asarray(level_boxes, np.int32).reshape(-1, 6))
    t = np.ascontiguousarray(np.asarray(tags, np.int32).reshape(-1, 3))
    f = None if carried is None else np.ascontiguousarray(np.asarray(carried, np.int32).reshape(-1, 3))
    cap = _cluster_cap(len(t) + (0 if f is None else len(f)))
    while True:
        out = np.empty((cap, 6), np.int32)
        nb = c_int32()
        if f is None:
            st = lib.sh_cluster_boxes(M, len(lb), lb.ctypes.data_as(c_void_p), blocking_factor, max_box,
                                      n_error_buf, efficiency, len(t), t.ctypes.data_as(c_void_p),
                                      out.ctypes.data_as(c_void_p), cap, ctypes.byref(nb))
        else:
            st = lib.sh_cluster_boxes_carried(M, len(lb), lb.ctypes.data_as(c_void_p), blocking_factor, max_box,
                                              n_error_buf, efficiency, len(t), t.ctypes.data_as(c_void_p), len(f),
                                              f.ctypes.data_as(c_void_p), grow, out.ctypes.data_as(c_void_p), cap,
                                              ctypes.byref(nb))
        if st == SH_ENOMEM and nb.value > cap:
            cap = nb.value
            continue
        _check(st)
        return [tuple(r) for r in out[:nb.value].tolist()]


def _cluster_cap(ntags: int) -> int:
    """First output capacity of a clustering call: a call whose boxes do not fit is run
    again with the count it reports, which clusters everything a second time, so the
    first buffer is sized from the tag count (a box holds at least one tag; in practice
    well under one box per 8 tags) and never below 65536 boxes (1.5 MiB, not touched
    beyond what is written)."""
    return max(1 << 16, ntags // 8)


def block_words(M: int, blocking_factor: int) -> int:
    """Words of the tagged-block bitset of a level of M cells per axis (blocks of bf/2)."""
    nb = M // (blocking_factor // 2)
    return (nb ** 3 + 63) // 64


def cluster_boxes_bits(M: int, level_boxes, bits, blocking_factor: int = 8, max_box: int = 64,
                       efficiency: float = 0.7):
    """Berger-Rigoutsos clustering from a tagged-block bitset (host only)."""
    lib = load()
    lb = np.ascontiguousarray(np.asarray(level_boxes, np.int32).reshape(-1, 6))
    bb = np.ascontiguousarray(bits, np.uint64)
    return _boxes_call(lambda out, cap, nb: lib.sh_cluster_boxes_bits(
        M, len(lb), lb.ctypes.data_as(c_void_p), blocking_factor, max_box, efficiency, bb.ctypes.data_as(c_void_p),
        len(bb), out, cap, nb))


def dilate_octants(M: int, octants, blocking_factor: int = 8, bits=None):
    """OR eight octant bitsets (shape (8, nwords)), each grown by one block towards its
    octant, into a block bitset (host only; sh_dilate_octants)."""
    lib = load()
    nw = block_words(M, blocking_factor)
    o = np.ascontiguousarray(octants, np.uint64).reshape(8, nw)
    out = np.zeros(nw, np.uint64) if bits is None else bits
    _check(lib.sh_dilate_octants(M, blocking_factor, o.ctypes.data_as(c_void_p), out.ctypes.data_as(c_void_p), nw))
    return out


def _boxes_call(fn):
    """Run a box-producing library call with a growing output capacity."""
    cap = 1 << 16
    while True:
        out = np.empty((cap, 6), np.int32)
        nb = c_int32()
        st = fn(out.ctypes.data_as(c_void_p), cap, ctypes.byref(nb))
        if st == SH_ENOMEM and nb.value > cap:
            cap = nb.value
            continue
        _check(st)
        return [tuple(r) for r in out[:nb.value].tolist()]


def local_tag_boxes(M_fine: int, fine_boxes, tags, blocking_factor: int = 8, n_error_buf: int = 2,
                    max_box: int = 64):
    """Boxes to add to a level (M_fine cells per axis) for the tags of the level below
    (local regrid, see sh_local_tag_boxes; host only)."""
    lib = load()
    fb = np.ascontiguousarray(np.asarray(fine_boxes, np.int32).reshape(-1, 6))
    t = np.ascontiguousarray(np.asarray(tags, np.int32).reshape(-1, 3))
    return _boxes_call(lambda out, cap, nb: lib.sh_local_tag_boxes(
        M_fine, len(fb), fb.ctypes.data_as(c_void_p), blocking_factor, n_error_buf, max_box, len(t),
        t.ctypes.data_as(c_void_p), out, cap, nb))


def local_nest_boxes(M_level: int, added_fine, level_boxes, blocking_factor: int = 8, max_box: int = 64):
    """Boxes to add to a level so that the added boxes of the next finer level keep their
    nesting gap (local regrid, see sh_local_nest_boxes; host only)."""
    lib = load()
    ab = np.ascontiguousarray(np.asarray(added_fine, np.int32).reshape(-1, 6))
    lb = np.ascontiguousarray(np.asarray(level_boxes, np.int32).reshape(-1, 6))
    return _boxes_call(lambda out, cap, nb: lib.sh_local_nest_boxes(
        M_level, len(ab), ab.ctypes.data_as(c_void_p), len(lb), lb.ctypes.data_as(c_void_p), blocking_factor,
        max_box, out, cap, nb))


def stream_probe(kind: int, src, dst, nbytes: int, stream):
    """One launch of the library's streaming probe (0 read, 1 write, 2 copy) of nbytes
    on `stream` (torch tensors as buffers)."""
    lib = load()
    _check(lib.sh_stream_probe(kind, c_void_p(src.data_ptr() if src is not None else 0),
                               c_void_p(dst.data_ptr()), nbytes, c_void_p(stream.cuda_stream)))


class Hierarchy:
    """One simulation: levels of boxes in caller-owned (torch) device arenas."""

    def __init__(self, n0: int, L: float, cfl: float = 0.25, eta0: float = 0.1, lam: float = 1.0,
                 alpha: float = 2.0, beta: int = 2, max_level: int = 0, blocking_factor: int = 8,
                 max_box: int = 64, n_error_buf: int = 2, prec: int = SH_F64, stream=None,
                 integrator: int = 4, lap_order: int = 1, interp: int = 1, ko_order: int = 0,
                 ko_eps: float = 0.0, tee_fields: int = 0):
        import torch
        self.torch = torch
        self.lib = load()
        self.params = sh_params(n0, L, cfl, eta0, lam, alpha, beta, max_level, blocking_factor, max_box,
                                n_error_buf, prec, integrator, lap_order, interp, ko_order, ko_eps,
                                int(tee_fields))
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = c_void_p()
        _check(self.lib.sh_hierarchy_create(ctypes.byref(self.params), c_void_p(self.stream.cuda_stream),
                                            ctypes.byref(h)))
        self.h = h
        self.arenas = {}
        self.boxes = {}
        self._tag_cap = {}

    # -- lifetime ---------------------------------------------------------------------
    def close(self):
        if self.h is not None:
            self.lib.sh_hierarchy_destroy(self.h)
            self.h = None
            self.arenas.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- layout -----------------------------------------------------------------------
    def arena_bytes(self, lev: int, boxes) -> int:
        b, ptr = _boxes_arr(boxes)
        n = self.lib.sh_arena_bytes(ctypes.byref(self.params), lev, len(b), ptr)
        if n == 0:
            raise ShError(SH_EINVAL, "invalid layout")
        return int(n)

    def set_layout(self, lev: int, boxes):
        b, ptr = _boxes_arr(boxes)
        if len(b) == 0:
            _check(self.lib.sh_set_level_layout(self.h, lev, 0, None, None, 0))
            for l in [k for k in self.arenas if k >= lev]:
                del self.arenas[l]
                del self.boxes[l]
            return
        nbytes = self.arena_bytes(lev, b)
        with self.torch.cuda.stream(self.stream):
            arena = self.torch.empty(nbytes, dtype=self.torch.uint8, device="cuda")
        _check(self.lib.sh_set_level_layout(self.h, lev, len(b), ptr, c_void_p(arena.data_ptr()), nbytes))
        self.arenas[lev] = arena  # the previous arena is released after the call (stream-ordered)
        self.boxes[lev] = [tuple(r) for r in b.tolist()]

    def num_levels(self) -> int:
        return int(self.lib.sh_num_levels(self.h))

    def level_info(self, lev: int):
        k, eta, nb, nc = c_int64(), c_double(), c_int32(), c_int64()
        _check(self.lib.sh_level_info(self.h, lev, ctypes.byref(k), ctypes.byref(eta), ctypes.byref(nb),
                                      ctypes.byref(nc)))
        return {"k": k.value, "eta": eta.value, "nboxes": nb.value, "ncells": nc.value}

    # -- state I/O --------------------------------------------------------------------
    def _count(self, lev, ghosts):
        g = 2 if ghosts else 0
        return sum(4 * (s[0] + g) * (s[1] + g) * (s[2] + g) for s in map(box_shape, self.boxes[lev]))

    def write_boxes(self, lev: int, arrays, role: int = ROLE_UN, ghosts: bool = False):
        """arrays: per-box (4, nz, ny, nx) float64 arrays (with the ghost shell if ghosts)."""
        flat = np.ascontiguousarray(np.concatenate([np.asarray(a, np.float64).ravel() for a in arrays]))
        if flat.size != self._count(lev, ghosts):
            raise ValueError("state size does not match the layout")
        _check(self.lib.sh_write_state(self.h, lev, role, flat.ctypes.data_as(c_void_p), 0, int(ghosts)))

    def read_boxes(self, lev: int, role: int = ROLE_UN, ghosts: bool = False):
        n = self._count(lev, ghosts)
        flat = np.empty(n, np.float64)
        _check(self.lib.sh_read_state(self.h, lev, role, flat.ctypes.data_as(c_void_p), 0, int(ghosts)))
        out, o = [], 0
        g = 2 if ghosts else 0
        for b in self.boxes[lev]:
            nz, ny, nx = box_shape(b)
            sz = 4 * (nz + g) * (ny + g) * (nx + g)
            out.append(flat[o:o + sz].reshape(4, nz + g, ny + g, nx + g))
            o += sz
        return out

    def read_device(self, lev: int, role: int = ROLE_UN):
        """Buffer `role` of level `lev` as a flat float64 device tensor in the dense box
        order (no ghosts), queued on the hierarchy's stream."""
        out = self.torch.empty(self._count(lev, False), dtype=self.torch.float64, device="cuda")
        _check(self.lib.sh_read_state(self.h, lev, role, c_void_p(out.data_ptr()), 1, 0))
        return out

    def write_device(self, lev: int, flat, role: int = ROLE_UN):
        """Write a float64 device tensor holding the level's boxes in the dense box order
        (no ghosts); queued on the hierarchy's stream, nothing allocated."""
        if flat.numel() != self._count(lev, False) or flat.dtype != self.torch.float64 or not flat.is_cuda:
            raise ValueError("state size, type or device does not match the layout")
        _check(self.lib.sh_write_state(self.h, lev, role, c_void_p(flat.data_ptr()), 1, 0))

    def write_dense(self, lev: int, U: np.ndarray, role: int = ROLE_UN):
        """Write a dense (4, M, M, M) level array (valid cells of each box are taken)."""
        arrs = []
        for b in self.boxes[lev]:
            arrs.append(U[:, b[2]:b[5] + 1, b[1]:b[4] + 1, b[0]:b[3] + 1])
        self.write_boxes(lev, arrs, role)

    def read_dense(self, lev: int, role: int = ROLE_UN, fill=np.nan) -> np.ndarray:
        M = self.params.n0 << lev
        U = np.full((4, M, M, M), fill)
        for b, a in zip(self.boxes[lev], self.read_boxes(lev, role)):
            U[:, b[2]:b[5] + 1, b[1]:b[4] + 1, b[0]:b[3] + 1] = a
        return U

    # -- the level step ---------------------------------------------------------------
    def fill_ghosts(self, lev: int, role: int = ROLE_UN, alpha_num: int = 4):
        _check(self.lib.sh_fill_ghosts(self.h, lev, role, alpha_num))

    def advance(self, lev: int, substep: int = 0):
        _check(self.lib.sh_advance_level(self.h, lev, substep))

    def average_down(self, fine_lev: int):
        _check(self.lib.sh_average_down(self.h, fine_lev))

    def tag(self, lev: int, want_idx: bool = True, mask_dev=None):
        """Tagged cells of a level: (count, (n, 3) int32 global x, y, z or None)."""
        n = c_int64()
        mptr = c_void_p(mask_dev.data_ptr()) if mask_dev is not None else None
        if not want_idx:
            _check(self.lib.sh_tag_cells(self.h, lev, mptr, None, 0, ctypes.byref(n)))
            return n.value, None
        # one call when the list fits the capacity remembered from this level's last
        # tagging (the count is always exact), a second one only when it grew past it
        cap = self._tag_cap.get(lev, 1 << 16)
        idx = np.empty((cap, 3), np.int32)
        _check(self.lib.sh_tag_cells(self.h, lev, mptr, idx.ctypes.data_as(c_void_p), cap, ctypes.byref(n)))
        if n.value > cap:
            cap = n.value + n.value // 4
            idx = np.empty((cap, 3), np.int32)
            _check(self.lib.sh_tag_cells(self.h, lev, mptr, idx.ctypes.data_as(c_void_p), cap, ctypes.byref(n)))
        self._tag_cap[lev] = max(cap, 1 << 16)
        return n.value, idx[:n.value]

    def tag_mask_dense(self, lev: int) -> np.ndarray:
        """Tag mask of a level as a dense uint8 (M, M, M) array (0 outside the level)."""
        torch = self.torch
        nv = sum(int(np.prod(box_shape(b))) for b in self.boxes[lev])
        m = torch.zeros(nv, dtype=torch.uint8, device="cuda")
        self.tag(lev, want_idx=False, mask_dev=m)
        mh = m.cpu().numpy()
        M = self.params.n0 << lev
        out = np.zeros((M, M, M), np.uint8)
        o = 0
        for b in self.boxes[lev]:
            nz, ny, nx = box_shape(b)
            out[b[2]:b[5] + 1, b[1]:b[4] + 1, b[0]:b[3] + 1] = mh[o:o + nz * ny * nx].reshape(nz, ny, nx)
            o += nz * ny * nx
        return out

    # -- truncation error estimates ---------------------------------------------------
    def set_tee(self, enable: bool = True, te_crit: float = 0.0, tag_mode: int = 3):
        """Compute estimates at every synchronisation; tag by plaquettes (1), by estimate
        above te_crit (2) or either (3)."""
        _check(self.lib.sh_set_tee(self.h, int(enable), float(te_crit), int(tag_mode)))

    def shadow_begin(self):
        _check(self.lib.sh_shadow_begin(self.h))

    def shadow_advance(self):
        _check(self.lib.sh_shadow_advance(self.h))

    def shadow_end(self):
        _check(self.lib.sh_shadow_end(self.h))

    def set_stream(self, stream):
        """Queue this hierarchy's later work on ``stream`` (see sh_set_stream); the arenas
        are marked as used there for torch's allocator."""
        _check(self.lib.sh_set_stream(self.h, c_void_p(stream.cuda_stream)))
        for a in self.arenas.values():
            a.record_stream(stream)
        self.stream = stream

    def restart(self):
        """Step counters back to 0 (see sh_restart)."""
        _check(self.lib.sh_restart(self.h))

    def set_debug(self, poison_ghosts: bool = True):
        """NaN into ghost shells before every complete fill (see sh_set_debug)."""
        _check(self.lib.sh_set_debug(self.h, 1 if poison_ghosts else 0))

    def set_tee_fields(self, enable: bool = True, te_crit=(0.0, 0.0, 0.0, 0.0), scale=None, tag_mode: int = 3):
        """Per-field thresholds and modifier scales (see sh_set_tee_fields)."""
        crit = (c_double * 4)(*[float(v) for v in te_crit])
        sc = (c_double * 4)(*[float(v) for v in scale]) if scale is not None else None
        _check(self.lib.sh_set_tee_fields(self.h, int(enable), crit, sc, int(tag_mode)))

    def field_absmax(self) -> np.ndarray:
        out = (c_double * 4)()
        _check(self.lib.sh_field_absmax(self.h, out))
        return np.array(list(out))

    def tee_dense(self, lev: int) -> np.ndarray:
        """A level's estimates as a dense float64 (M, M, M) array, or (4, M, M, M) with one
        estimate per component (0 outside the level)."""
        torch = self.torch
        nc = 4 if self.params.tee_fields else 1
        nv = sum(int(np.prod(box_shape(b))) for b in self.boxes[lev])
        with torch.cuda.stream(self.stream):
            t = torch.empty(max(nc * nv, 1), dtype=torch.float64, device="cuda")
        _check(self.lib.sh_read_tee(self.h, lev, c_void_p(t.data_ptr())))
        th = t.cpu().numpy()[:nc * nv].reshape(nc, max(nv, 0))
        M = self.params.n0 << lev
        out = np.zeros((nc, M, M, M))
        o = 0
        for b in self.boxes[lev]:
            nz, ny, nx = box_shape(b)
            out[:, b[2]:b[5] + 1, b[1]:b[4] + 1, b[0]:b[3] + 1] = th[:, o:o + nz * ny * nx].reshape(nc, nz, ny, nx)
            o += nz * ny * nx
        return out if nc == 4 else out[0]

    def energy(self):
        e = (c_double * 4)()
        bad = c_int64()
        _check(self.lib.sh_energy(self.h, e, ctypes.byref(bad)))
        return list(e), bad.value

    def eval_rhs(self, lev: int):
        torch = self.torch
        n = self._count(lev, False)
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        _check(self.lib.sh_eval_rhs(self.h, lev, c_void_p(out.data_ptr())))
        self.sync()
        flat = out.cpu().numpy()
        res, o = [], 0
        for b in self.boxes[lev]:
            nz, ny, nx = box_shape(b)
            sz = 4 * nz * ny * nx
            res.append(flat[o:o + sz].reshape(4, nz, ny, nx))
            o += sz
        return res

    def tag_blocks(self, lev: int, r: int, halve: bool = False, bits=None):
        """Tag a level on the GPU and OR the blocks its tagged cells, grown by r, meet into
        a block bitset of that level (of the level below with ``halve``, from the cells'
        parents): (tag count, uint64 bitset).  See sh_tag_blocks."""
        M = (self.params.n0 << lev) >> (1 if halve else 0)
        nw = block_words(M, self.params.blocking_factor)
        out = np.zeros(nw, np.uint64) if bits is None else bits
        n = c_int64()
        _check(self.lib.sh_tag_blocks(self.h, lev, int(halve), r, out.ctypes.data_as(c_void_p), nw, ctypes.byref(n)))
        return n.value, out

    def cluster_blocks(self, lev: int, bits, efficiency: float = 0.7):
        """Boxes of level lev+1 from a bitset of level lev's tagged blocks (sh_cluster_blocks)."""
        bb = np.ascontiguousarray(bits, np.uint64)
        return _boxes_call(lambda out, cap, nb: self.lib.sh_cluster_blocks(
            self.h, lev, bb.ctypes.data_as(c_void_p), len(bb), efficiency, out, cap, nb))

    def cluster(self, lev: int, tags: np.ndarray, efficiency: float = 0.7, carried=None, grow: int = 1):
        """Boxes of level lev+1 from level lev's tags (sh_cluster_tags); with ``carried``,
        tags of level lev+1 join through their grown coarse parents (sh_cluster_tags_carried)."""
        t = np.ascontiguousarray(np.asarray(tags, np.int32).reshape(-1, 3))
        f = None if carried is None else np.ascontiguousarray(np.asarray(carried, np.int32).reshape(-1, 3))
        cap = _cluster_cap(len(t) + (0 if f is None else len(f)))
        while True:
            out = np.empty((cap, 6), np.int32)
            nb = c_int32()
            if f is None:
                st = self.lib.sh_cluster_tags(self.h, lev, len(t), t.ctypes.data_as(c_void_p), efficiency,
                                              out.ctypes.data_as(c_void_p), cap, ctypes.byref(nb))
            else:
                st = self.lib.sh_cluster_tags_carried(self.h, lev, len(t), t.ctypes.data_as(c_void_p), len(f),
                                                      f.ctypes.data_as(c_void_p), grow, efficiency,
                                                      out.ctypes.data_as(c_void_p), cap, ctypes.byref(nb))
            if st == SH_ENOMEM and nb.value > cap:
                cap = nb.value
                continue
            _check(st)
            return [tuple(r) for r in out[:nb.value].tolist()]

    def sync(self):
        _check(self.lib.sh_sync(self.h))

    def stage_scalars(self, lev: int, s: int):
        out = (c_double * 7)()
        _check(self.lib.sh_debug_stage_scalars(self.h, lev, s, out))
        return list(out)

    def set_tuning(self, kind: int = 8, nontemporal: int = 1, tile_z: int = 0, fuse: int = 4,
                   fused_shape: int | None = None, fused_tile_z: int = 0, fused_variant: int | None = None):
        """Launch shape (see sh_set_tuning); the fused shape and variant default to the
        library's choice for the hierarchy's precision."""
        ssp = self.params.integrator in (3, 10)
        if fused_shape is None:
            fused_shape = 2
        if fused_variant is None:
            fused_variant = 5 if ssp else (6 if self.params.prec == SH_F32 else 3)
        _check(self.lib.sh_set_tuning(self.h, kind, nontemporal, tile_z, fuse, fused_shape, fused_tile_z,
                                      fused_variant))

    def capture(self):
        """``with h.capture() as c: driver.coarse_step(h)`` records the level steps issued
        inside the block (they do not run); ``c.graph.launch()`` replays them."""
        return _Capture(self)

    PROFILE_CLASSES = ("stage1", "stage2", "stage3", "stage4", "ghost_copy", "ghost_interp",
                       "average_down", "fused_step")

    def profile(self, enable: bool):
        _check(self.lib.sh_profile(self.h, int(enable)))

    def profile_read(self):
        """{class: (total_ms, launches)} of the launches timed since profile(True)."""
        ms = (c_double * 8)()
        n = (c_int64 * 8)()
        _check(self.lib.sh_profile_read(self.h, ms, n))
        return {c: (ms[i], n[i]) for i, c in enumerate(self.PROFILE_CLASSES)}

    def trace(self, enable: bool):
        _check(self.lib.sh_trace(self.h, int(enable)))

    def trace_read(self):
        n = self.lib.sh_trace_read(self.h, None, 0)
        buf = np.empty((max(n, 1), 4), np.int32)
        self.lib.sh_trace_read(self.h, buf.ctypes.data_as(c_void_p), n)
        return [tuple(r) for r in buf[:n].tolist()]


class Batch:
    """One RK4 step of many single-level hierarchies per launch (see sh_batch_create)."""

    def __init__(self, hierarchies):
        self.lib = load()
        self.members = list(hierarchies)
        arr = (c_void_p * len(self.members))(*[m.h.value for m in self.members])
        b = c_void_p()
        _check(self.lib.sh_batch_create(len(self.members), arr, ctypes.byref(b)))
        self.b = b

    def advance(self):
        _check(self.lib.sh_batch_advance(self.b))

    def update(self, hierarchies):
        """New members, same device tables (see sh_batch_update)."""
        self.members = list(hierarchies)
        arr = (c_void_p * len(self.members))(*[m.h.value for m in self.members])
        _check(self.lib.sh_batch_update(self.b, len(self.members), arr))

    def capture(self, nsteps: int) -> "Graph":
        """Record ``nsteps`` batch steps as one replayable graph (see sh_batch_capture)."""
        g = c_void_p()
        _check(self.lib.sh_batch_capture(self.b, nsteps, ctypes.byref(g)))
        return Graph(g)

    def close(self):
        if self.b is not None:
            self.lib.sh_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A recorded sequence of level steps; ``launch()`` replays it on the recording stream."""

    def __init__(self, g):
        self.lib = load()
        self.g = g

    def launch(self):
        _check(self.lib.sh_graph_launch(self.g))

    def close(self):
        if self.g is not None:
            self.lib.sh_graph_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Capture:
    def __init__(self, h):
        self.h = h
        self.graph = None

    def __enter__(self):
        _check(self.h.lib.sh_capture_begin(self.h.h))
        return self

    def __exit__(self, exc_type, exc, tb):
        g = c_void_p()
        st = self.h.lib.sh_capture_end(self.h.h, ctypes.byref(g))
        if exc_type is None:
            _check(st)
            self.graph = Graph(g)
        elif g.value:
            self.h.lib.sh_graph_destroy(g)
        return False

