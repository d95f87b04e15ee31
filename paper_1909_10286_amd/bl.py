"""ctypes binding of libbl.so (include/bl.h), argument marshalling only.

Every step of the evaluation runs in the library's HIP kernels; PyTorch only
provides device buffers (``tensor.data_ptr()``) and the stream.  Loading fails
loudly when the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import List, Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libbl.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, EINFEASIBLE = 0, -1, -2, -3, -4, -5
FIXED_FIELD_BP, NO_EMBEDDED_MIN, GATE_OFF, GATE_STRICT, FULL_WALK, WIDE_KEYS, SEGMENT_EVAL = (
    1, 2, 4, 8, 16, 32, 64)
TIMING_EVAL = 1
TIMING_SCREEN = 2
CAND_INFEASIBLE, CAND_GATED, CAND_CAP_HU, CAND_CAP_SU, CAND_INVALID, CAND_INF_MAKESPAN = (
    1, 2, 4, 8, 16, 32)
SLOT_BASE, SLOT_BEST, SLOT_OLD = 0, 1, 2
INF_KEY = (1 << 64) - 1
INF_MAKESPAN = 0x7FFFFFFF

_u32p = C.POINTER(C.c_uint32)
_u16p = C.POINTER(C.c_uint16)
_i32p = C.POINTER(C.c_int32)


class _Instance(C.Structure):
    _fields_ = [("n_fields", C.c_int32), ("n_bps", C.c_int32), ("n_tours", C.c_int32),
                ("n_hus", C.c_int32), ("n_sus", C.c_int32),
                ("dist_m", _u32p), ("field_area", _u32p), ("field_yield", _u32p),
                ("bp_demand_kg", _u32p), ("hu_rate", _u32p), ("hu_speed_mph", C.c_uint32),
                ("su_cap_kg", _u32p), ("su_speed_mph", _u32p), ("su_fill_s", _u32p),
                ("xy_m", _i32p), ("init_hus_per_tour", _u16p), ("init_sus_per_tour", _u16p),
                ("flags", C.c_uint32), ("cap_hu", C.c_uint32), ("cap_su", C.c_uint32)]


class _Solution(C.Structure):
    _fields_ = [("tour_off", _u16p), ("tour_bp", _u16p), ("bp_off", _u16p),
                ("bp_field", _u16p), ("hu_tour", _u16p), ("su_tour", _u16p)]


class _SearchParams(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("eps_threshold", C.c_uint64), ("n", C.c_uint32),
                ("inst_index", C.c_uint32)]


class _SearchState(C.Structure):
    _fields_ = [("it", C.c_uint32), ("n_improved", C.c_uint32), ("cost_best_m", C.c_uint64),
                ("t_best_s", C.c_int64)]


class _InstanceInfo(C.Structure):
    _fields_ = [("lane_eval", C.c_int32), ("tail_table", C.c_int32), ("wg_per_cu", C.c_int32),
                ("image_bytes", C.c_uint32)]


class _SurConfig(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("adam_eps", C.c_float),
                ("max_examples", C.c_uint32), ("c0_m", C.c_float), ("t0_s", C.c_float)]


class _ScreenParams(C.Structure):
    _fields_ = [("n_proposals", C.c_uint32), ("n_shortlist", C.c_uint32), ("n_fallback", C.c_uint32),
                ("mk_margin", C.c_float), ("err_threshold", C.c_float), ("n_control", C.c_uint32)]


class _SurStats(C.Structure):
    _fields_ = [("iterations", C.c_uint32), ("fallbacks", C.c_uint32), ("last_used", C.c_uint32),
                ("last_error", C.c_float)]


class _Schedule(C.Structure):
    _fields_ = [("tile", C.c_uint32 * 3), ("order_policy", C.c_uint32), ("feas_queue", C.c_uint32)]


class _TraceRow(C.Structure):
    _fields_ = [("best_key", C.c_uint64), ("cost_m", C.c_uint64), ("makespan_s", C.c_int64),
                ("it", C.c_uint32), ("indicator", C.c_uint8), ("use_best", C.c_uint8),
                ("pad", C.c_uint8 * 2)]


_SIGS = {
    "bl_create": (C.c_int32, [C.c_int32, C.POINTER(C.c_void_p)]),
    "bl_destroy": (None, [C.c_void_p]),
    "bl_set_stream": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "bl_status_str": (C.c_char_p, [C.c_int32]),
    "bl_last_error": (C.c_char_p, [C.c_void_p]),
    "bl_instance_upload": (C.c_int32, [C.c_void_p, C.POINTER(_Instance), C.POINTER(C.c_int32)]),
    "bl_instance_info_get": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(_InstanceInfo)]),
    "bl_init_solution": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(_Solution)]),
    "bl_solution_upload": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(_Solution)]),
    "bl_solution_download": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(_Solution)]),
    "bl_generate": (C.c_int32, [C.c_void_p, C.c_int32, C.c_uint64, C.c_uint32, C.c_uint32,
                                C.c_uint32, C.c_uint32, C.c_void_p]),
    "bl_evaluate_batch": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_uint32, C.c_int64,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "bl_evaluate_batch_static": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_uint32, C.c_int64,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "bl_select_best": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p]),
    "bl_search_start": (C.c_int32, [C.c_void_p, C.c_int32, C.c_uint32]),
    "bl_search_step": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(_SearchParams)]),
    "bl_search_state_get": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(_SearchState)]),
    "bl_search_trace": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(_TraceRow), C.c_uint32,
                                    C.POINTER(C.c_uint32)]),
    "bl_batch_create": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.c_int32, C.c_uint32,
                                    C.POINTER(C.c_int32)]),
    "bl_batch_start": (C.c_int32, [C.c_void_p, C.c_int32, C.c_uint32]),
    "bl_batch_step": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(_SearchParams)]),
    "bl_batch_set_schedule": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(_Schedule)]),
    "bl_batch_autotune": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(_SearchParams), C.c_char_p,
                                      C.POINTER(_Schedule)]),
    "bl_search_capture": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(_SearchParams), C.c_uint32,
                                      C.POINTER(C.c_int32)]),
    "bl_batch_capture": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(_SearchParams), C.c_uint32,
                                     C.POINTER(C.c_int32)]),
    "bl_graph_launch": (C.c_int32, [C.c_void_p, C.c_int32]),
    "bl_sur_create": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_float), C.POINTER(_SurConfig),
                                  C.POINTER(C.c_int32)]),
    "bl_sur_get_weights": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_float)]),
    "bl_sur_set_weights": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_float)]),
    "bl_sur_predict": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_uint32, C.c_void_p]),
    "bl_sur_gradients": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_uint32, C.POINTER(C.c_float), C.POINTER(C.c_double)]),
    "bl_sur_train_step": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_uint32, C.c_void_p]),
    "bl_sur_screen": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(_SearchParams),
                                  C.POINTER(_ScreenParams), C.c_void_p, C.c_void_p]),
    "bl_sur_search_step": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(_SearchParams),
                                       C.POINTER(_ScreenParams)]),
    "bl_sur_stats_get": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(_SurStats)]),
    "bl_timing_enable": (C.c_int32, [C.c_void_p, C.c_int32]),
    "bl_timing_read": (C.c_int32, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_uint32)]),
    "bl_measure_peaks": (C.c_int32, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
}

EXPORTED = sorted(_SIGS)
_lib: Optional[C.CDLL] = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libbl.so and declare its signatures; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libbl.so is not built (%s); run __graft_entry__.build()" % path)
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class BlError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s (%d): %s" % (load().bl_status_str(status).decode(), status, msg))
        self.status = status


@dataclasses.dataclass
class CSR:
    """Solution in the library's compressed-list layout (numpy uint16)."""
    tour_off: np.ndarray
    tour_bp: np.ndarray
    bp_off: np.ndarray
    bp_field: np.ndarray
    hu_tour: np.ndarray
    su_tour: np.ndarray

    @staticmethod
    def empty(nf, nb, nt, nhu, nsu) -> "CSR":
        z = lambda n: np.zeros(n, dtype=np.uint16)
        return CSR(z(nt + 1), z(nb), z(nb + 1), z(nf), z(nhu), z(nsu))

    @staticmethod
    def from_lists(tours: List[List[int]], fields: List[List[int]], hu_tour, su_tour) -> "CSR":
        toff = np.cumsum([0] + [len(t) for t in tours]).astype(np.uint16)
        boff = np.cumsum([0] + [len(f) for f in fields]).astype(np.uint16)
        cat = lambda xs: np.asarray([v for x in xs for v in x], dtype=np.uint16)
        return CSR(toff, cat(tours), boff, cat(fields), np.asarray(hu_tour, np.uint16),
                   np.asarray(su_tour, np.uint16))

    def to_lists(self):
        t = [list(map(int, self.tour_bp[self.tour_off[g]:self.tour_off[g + 1]]))
             for g in range(len(self.tour_off) - 1)]
        f = [list(map(int, self.bp_field[self.bp_off[b]:self.bp_off[b + 1]]))
             for b in range(len(self.bp_off) - 1)]
        return t, f, list(map(int, self.hu_tour)), list(map(int, self.su_tour))

    def _struct(self) -> _Solution:
        for a in (self.tour_off, self.tour_bp, self.bp_off, self.bp_field, self.hu_tour, self.su_tour):
            assert a.dtype == np.uint16 and a.flags.c_contiguous
        p = lambda a: a.ctypes.data_as(_u16p)
        return _Solution(p(self.tour_off), p(self.tour_bp), p(self.bp_off), p(self.bp_field),
                         p(self.hu_tour), p(self.su_tour))


def _ptr(t) -> int:
    """Device pointer of a torch tensor (or an int already), or NULL."""
    if t is None:
        return 0
    if isinstance(t, int):
        return t
    return int(t.data_ptr())


class Context:
    """One library context on one GPU.  Methods mirror the C calls."""

    def __init__(self, device: int = 0):
        self._lib = load()
        h = C.c_void_p()
        st = self._lib.bl_create(device, C.byref(h))
        if st != OK:
            raise BlError(st, "bl_create(%d)" % device)
        self._h = h
        self._sizes = {}

    def close(self):
        if self._h:
            self._lib.bl_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != OK:
            raise BlError(st, self._lib.bl_last_error(self._h).decode())

    def set_stream(self, stream):
        """stream: torch.cuda.Stream, a raw hipStream_t int, or None (default)."""
        raw = 0 if stream is None else (stream if isinstance(stream, int) else stream.cuda_stream)
        self._check(self._lib.bl_set_stream(self._h, C.c_void_p(raw)))

    def instance_upload(self, inst, flags: int = 0, cap_hu: int = 0, cap_su: int = 0) -> int:
        keep = []

        def u32(a):
            a = np.ascontiguousarray(a, dtype=np.uint32)
            keep.append(a)
            return a.ctypes.data_as(_u32p)

        def u16(a):
            if a is None:
                return C.cast(None, _u16p)
            a = np.ascontiguousarray(a, dtype=np.uint16)
            keep.append(a)
            return a.ctypes.data_as(_u16p)
        xy = np.ascontiguousarray(np.asarray(inst.xy_m).reshape(-1), dtype=np.int32)
        keep.append(xy)
        s = _Instance(inst.n_fields, inst.n_bps, inst.n_tours, inst.n_hus, inst.n_sus,
                      u32(inst.dist_m), u32(inst.field_area), u32(inst.field_yield),
                      u32(inst.bp_demand_kg), u32(inst.hu_rate), int(inst.hu_speed_mph),
                      u32(inst.su_cap_kg), u32(inst.su_speed_mph), u32(inst.su_fill_s),
                      xy.ctypes.data_as(_i32p), u16(inst.init_hus_per_tour),
                      u16(inst.init_sus_per_tour), flags, cap_hu, cap_su)
        out = C.c_int32()
        self._check(self._lib.bl_instance_upload(self._h, C.byref(s), C.byref(out)))
        self._sizes[out.value] = (inst.n_fields, inst.n_bps, inst.n_tours, inst.n_hus, inst.n_sus)
        return out.value

    def init_solution(self, inst_id: int) -> CSR:
        sol = CSR.empty(*self._sizes[inst_id])
        self._check(self._lib.bl_init_solution(self._h, inst_id, C.byref(sol._struct())))
        return sol

    def solution_upload(self, inst_id: int, slot: int, sol: CSR):
        self._check(self._lib.bl_solution_upload(self._h, inst_id, slot, C.byref(sol._struct())))

    def solution_download(self, inst_id: int, slot: int) -> CSR:
        sol = CSR.empty(*self._sizes[inst_id])
        self._check(self._lib.bl_solution_download(self._h, inst_id, slot, C.byref(sol._struct())))
        return sol

    def generate(self, inst_id, seed, it, inst_index, first, n, d_moves):
        self._check(self._lib.bl_generate(self._h, inst_id, seed, it, inst_index, first, n,
                                          C.c_void_p(_ptr(d_moves))))

    def evaluate_batch(self, inst_id, d_moves, n, t_star_s, d_key, d_cost=None, d_makespan=None,
                       d_flags=None):
        self._check(self._lib.bl_evaluate_batch(
            self._h, inst_id, C.c_void_p(_ptr(d_moves)), n, int(t_star_s),
            C.c_void_p(_ptr(d_key)), C.c_void_p(_ptr(d_cost)), C.c_void_p(_ptr(d_makespan)),
            C.c_void_p(_ptr(d_flags))))

    def evaluate_batch_static(self, inst_id, d_moves, n, t_star_s, d_key, d_cost=None, d_makespan=None,
                              d_flags=None):
        self._check(self._lib.bl_evaluate_batch_static(
            self._h, inst_id, C.c_void_p(_ptr(d_moves)), n, int(t_star_s),
            C.c_void_p(_ptr(d_key)), C.c_void_p(_ptr(d_cost)), C.c_void_p(_ptr(d_makespan)),
            C.c_void_p(_ptr(d_flags))))

    def select_best(self, d_key, n, d_best):
        self._check(self._lib.bl_select_best(self._h, C.c_void_p(_ptr(d_key)), n,
                                             C.c_void_p(_ptr(d_best))))

    def search_start(self, inst_id: int, trace_capacity: int = 0):
        self._check(self._lib.bl_search_start(self._h, inst_id, trace_capacity))

    def search_step(self, inst_id: int, seed: int, eps_threshold: int, n: int, inst_index: int = 0):
        p = _SearchParams(seed, eps_threshold, n, inst_index)
        self._check(self._lib.bl_search_step(self._h, inst_id, C.byref(p)))

    def instance_info(self, inst_id: int) -> dict:
        """How the instance is evaluated (bl_instance_info_get)."""
        s = _InstanceInfo()
        self._check(self._lib.bl_instance_info_get(self._h, inst_id, C.byref(s)))
        return dict(lane_eval=s.lane_eval, tail_table=s.tail_table, wg_per_cu=s.wg_per_cu,
                    image_bytes=s.image_bytes)

    def search_state(self, inst_id: int) -> dict:
        s = _SearchState()
        self._check(self._lib.bl_search_state_get(self._h, inst_id, C.byref(s)))
        return dict(it=s.it, n_improved=s.n_improved, cost_best_m=s.cost_best_m, t_best_s=s.t_best_s)

    def search_trace(self, inst_id: int, max_rows: int = 1 << 20) -> list:
        st = self.search_state(inst_id)
        rows = min(max_rows, st["it"])
        buf = (_TraceRow * max(rows, 1))()
        got = C.c_uint32()
        self._check(self._lib.bl_search_trace(self._h, inst_id, buf, rows, C.byref(got)))
        return [dict(best_key=r.best_key, cost_m=r.cost_m, makespan_s=r.makespan_s, it=r.it,
                     indicator=r.indicator, use_best=r.use_best) for r in buf[:got.value]]

    def timing_enable(self, on: bool = True, kind: int = None):
        """Time launches of the evaluation kernel (kind TIMING_EVAL, the
        default) or of the screen's scoring kernel (TIMING_SCREEN)."""
        kind = TIMING_EVAL if kind is None else kind
        self._check(self._lib.bl_timing_enable(self._h, kind if on else 0))

    def measure_peaks(self):
        """(HBM GB/s from a streaming copy, LDS GB/s from ds_read_b128 streams)."""
        h, l = C.c_double(), C.c_double()
        self._check(self._lib.bl_measure_peaks(self._h, C.byref(h), C.byref(l)))
        return h.value, l.value

    def timing_read(self):
        """(summed kernel ms, launches) of the timed kind since the last read."""
        ms, n = C.c_double(), C.c_uint32()
        self._check(self._lib.bl_timing_read(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    # ---------------------------------------------------------- batches --
    def batch_create(self, inst_ids, n_cand: int) -> int:
        ids = (C.c_int32 * len(inst_ids))(*inst_ids)
        out = C.c_int32()
        self._check(self._lib.bl_batch_create(self._h, ids, len(inst_ids), n_cand, C.byref(out)))
        return out.value

    def batch_start(self, batch: int, trace_capacity: int = 0):
        self._check(self._lib.bl_batch_start(self._h, batch, trace_capacity))

    def batch_step(self, batch: int, seed: int, eps_threshold: int, inst_index: int = 0):
        p = _SearchParams(seed, eps_threshold, 0, inst_index)
        self._check(self._lib.bl_batch_step(self._h, batch, C.byref(p)))

    def batch_set_schedule(self, batch: int, tiles, order_policy: int, feas_queue: int = 1):
        s = _Schedule((C.c_uint32 * 3)(*tiles), order_policy, feas_queue)
        self._check(self._lib.bl_batch_set_schedule(self._h, batch, C.byref(s)))

    def batch_autotune(self, batch: int, seed: int, eps_threshold: int, cache_path=None,
                       inst_index: int = 0) -> dict:
        p = _SearchParams(seed, eps_threshold, 0, inst_index)
        s = _Schedule()
        path = None if cache_path is None else os.fsencode(cache_path)
        self._check(self._lib.bl_batch_autotune(self._h, batch, C.byref(p), path, C.byref(s)))
        return dict(tile=list(s.tile), order_policy=s.order_policy, feas_queue=s.feas_queue)

    # ----------------------------------------------------------- graphs --
    def search_capture(self, inst_id: int, seed: int, eps_threshold: int, n: int, n_steps: int,
                       inst_index: int = 0) -> int:
        p = _SearchParams(seed, eps_threshold, n, inst_index)
        g = C.c_int32()
        self._check(self._lib.bl_search_capture(self._h, inst_id, C.byref(p), n_steps, C.byref(g)))
        return g.value

    def batch_capture(self, batch: int, seed: int, eps_threshold: int, n_steps: int,
                      inst_index: int = 0) -> int:
        p = _SearchParams(seed, eps_threshold, 0, inst_index)
        g = C.c_int32()
        self._check(self._lib.bl_batch_capture(self._h, batch, C.byref(p), n_steps, C.byref(g)))
        return g.value

    def graph_launch(self, graph: int):
        self._check(self._lib.bl_graph_launch(self._h, graph))

    # ---------------------------------------------------- learned screen --
    def sur_create(self, inst_id: int, weights, c0_m: float, t0_s: float, max_examples: int = 4096,
                   lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                   adam_eps: float = 1e-8) -> int:
        w = np.ascontiguousarray(weights, dtype=np.float32)
        assert w.size == SUR_PARAMS
        cfg = _SurConfig(lr, beta1, beta2, adam_eps, max_examples, c0_m, t0_s)
        out = C.c_int32()
        self._check(self._lib.bl_sur_create(self._h, inst_id, w.ctypes.data_as(C.POINTER(C.c_float)),
                                            C.byref(cfg), C.byref(out)))
        return out.value

    def sur_get_weights(self, sur: int) -> np.ndarray:
        w = np.empty(SUR_PARAMS, dtype=np.float32)
        self._check(self._lib.bl_sur_get_weights(self._h, sur, w.ctypes.data_as(C.POINTER(C.c_float))))
        return w

    def sur_set_weights(self, sur: int, weights):
        w = np.ascontiguousarray(weights, dtype=np.float32)
        self._check(self._lib.bl_sur_set_weights(self._h, sur, w.ctypes.data_as(C.POINTER(C.c_float))))

    def sur_predict(self, sur: int, d_moves, n: int, d_out):
        self._check(self._lib.bl_sur_predict(self._h, sur, C.c_void_p(_ptr(d_moves)), n,
                                             C.c_void_p(_ptr(d_out))))

    def sur_gradients(self, sur: int, d_moves, d_cost, d_mk, n: int):
        g = np.empty(SUR_PARAMS, dtype=np.float32)
        loss = C.c_double()
        self._check(self._lib.bl_sur_gradients(
            self._h, sur, C.c_void_p(_ptr(d_moves)), C.c_void_p(_ptr(d_cost)), C.c_void_p(_ptr(d_mk)), n,
            g.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss)))
        return g, loss.value

    def sur_train_step(self, sur: int, d_moves, d_cost, d_mk, n: int, d_loss=None):
        self._check(self._lib.bl_sur_train_step(
            self._h, sur, C.c_void_p(_ptr(d_moves)), C.c_void_p(_ptr(d_cost)), C.c_void_p(_ptr(d_mk)), n,
            C.c_void_p(_ptr(d_loss))))

    def sur_screen(self, sur: int, seed: int, eps_threshold: int, n_proposals: int, n_shortlist: int,
                   d_shortlist, d_score=None, mk_margin: float = 0.0, inst_index: int = 0):
        p = _SearchParams(seed, eps_threshold, 0, inst_index)
        sc = _ScreenParams(n_proposals, n_shortlist, 0, mk_margin, 0.0, 0)
        self._check(self._lib.bl_sur_screen(self._h, sur, C.byref(p), C.byref(sc),
                                            C.c_void_p(_ptr(d_shortlist)), C.c_void_p(_ptr(d_score))))

    def sur_search_step(self, sur: int, seed: int, eps_threshold: int, n_proposals: int,
                        n_shortlist: int, n_fallback: int, mk_margin: float = 0.0,
                        err_threshold: float = 0.05, n_control: int = 0, inst_index: int = 0):
        p = _SearchParams(seed, eps_threshold, 0, inst_index)
        sc = _ScreenParams(n_proposals, n_shortlist, n_fallback, mk_margin, err_threshold, n_control)
        self._check(self._lib.bl_sur_search_step(self._h, sur, C.byref(p), C.byref(sc)))

    def sur_stats(self, sur: int) -> dict:
        s = _SurStats()
        self._check(self._lib.bl_sur_stats_get(self._h, sur, C.byref(s)))
        return dict(iterations=s.iterations, fallbacks=s.fallbacks, last_used=s.last_used,
                    last_error=s.last_error)


SUR_PARAMS = 27586
SUR_SHAPES = [("W1", (16, 128)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)),
              ("W3", (136, 64)), ("b3", (64,)), ("W4", (64, 2)), ("b4", (2,))]


def sur_glorot_weights(draws) -> np.ndarray:
    """Initial weights in the library's order from uniform [0, 1) draws
    (W1, W2, W3, W4 draws in that order): Glorot-uniform weights, zero
    biases."""
    out, k = [], 0
    for name, shape in SUR_SHAPES:
        n = int(np.prod(shape))
        if name.startswith("W"):
            lim = np.sqrt(6.0 / (shape[0] + shape[1]))
            out.append((np.asarray(draws[k:k + n], dtype=np.float64) * 2 - 1) * lim)
            k += n
        else:
            out.append(np.zeros(n))
    return np.concatenate([o.reshape(-1) for o in out]).astype(np.float32)
