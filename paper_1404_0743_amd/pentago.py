"""Thin Python binding of the C ABI in include/pentago.h (argument marshalling
only: every step of the computation runs in the HIP library).

Device buffers are torch tensors on the current CUDA (HIP) device; the stream
is torch's current stream unless one is given.  The library must have been
built (``paper_1404_0743_amd.build.build()``); loading fails loudly otherwise.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpentago.so")

OK, EINVAL, ENOCHILD, ENOMEM, ERANGE, EAGAIN, EDEVICE = 0, -1, -2, -3, -4, -5, -6


class PentagoError(RuntimeError):
    def __init__(self, code, func, detail):
        super().__init__("%s failed: %s (%d): %s" % (func, _strerror(code), code, detail))
        self.code = code


class TileShape(ctypes.Structure):
    _fields_ = [("lines", ctypes.c_int32), ("threads", ctypes.c_int32), ("order", ctypes.c_int32)]


class Section(ctypes.Structure):
    _fields_ = [("black", ctypes.c_uint8 * 4), ("white", ctypes.c_uint8 * 4)]


class Board(ctypes.Structure):
    _fields_ = [("q", ctypes.c_uint16 * 4)]


class Set256(ctypes.Structure):
    _fields_ = [("w", ctypes.c_uint64 * 4)]


class SectionJob(ctypes.Structure):
    _fields_ = [("section", Section), ("child", ctypes.c_void_p * 4), ("out", ctypes.c_void_p)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("memory_budget", ctypes.c_uint64), ("max_inflight", ctypes.c_uint32),
                ("max_batch", ctypes.c_uint32), ("streams", ctypes.c_uint32)]


class ServeStats(ctypes.Structure):
    _fields_ = [("queries", ctypes.c_uint64), ("lookups", ctypes.c_uint64),
                ("searches", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("queries_per_s", ctypes.c_double),
                ("lookup_p50_us", ctypes.c_double), ("lookup_p99_us", ctypes.c_double),
                ("search_p50_us", ctypes.c_double), ("search_p99_us", ctypes.c_double)]


_lib = None

# name -> (argtypes, restype)
_P = ctypes.c_void_p
_SIGS = {
    "pentago_section_shape": ([Section, _P, _P, _P], ctypes.c_int),
    "pentago_section_offset": ([Section, _P, _P], ctypes.c_int),
    "pentago_section_board": ([Section, _P, _P], ctypes.c_int),
    "pentago_child_section": ([Section, ctypes.c_int, _P], ctypes.c_int),
    "pentago_solve_section": ([Section, _P, _P, _P], ctypes.c_int),
    "pentago_section_image": ([Section, ctypes.c_int, _P], ctypes.c_int),
    "pentago_section_standardize": ([Section, _P, _P], ctypes.c_int),
    "pentago_section_transform": ([Section, _P, ctypes.c_int, _P, _P], ctypes.c_int),
    "pentago_solve_section_d4": ([Section, _P, _P, _P], ctypes.c_int),
    "pentago_solve_sections": ([_P, ctypes.c_size_t, _P], ctypes.c_int),
    "pentago_solve_sections_d4": ([_P, ctypes.c_size_t, _P], ctypes.c_int),
    "pentago_plan_create_d4": ([_P, ctypes.c_size_t, _P], ctypes.c_int),
    "pentago_slice_sections": ([ctypes.c_int, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "pentago_autotune_section": ([Section, _P, _P, _P, _P, _P], ctypes.c_int),
    "pentago_solve_section_shape": ([Section, _P, _P, _P, _P], ctypes.c_int),
    "pentago_plan_create": ([_P, ctypes.c_size_t, _P], ctypes.c_int),
    "pentago_plan_launch": ([_P, _P], ctypes.c_int),
    "pentago_plan_launch_graph": ([_P, _P], ctypes.c_int),
    "pentago_plan_info": ([_P, _P, _P, _P], ctypes.c_int),
    "pentago_plan_destroy": ([_P], ctypes.c_int),
    "pentago_eval_batch": ([_P, ctypes.c_size_t, _P, _P, _P], ctypes.c_int),
    "pentago_eval_deep": ([Board, _P, _P], ctypes.c_int),
    "pentago_eval_deep_parity": ([Board, ctypes.c_int, _P, _P], ctypes.c_int),
    "pentago_eval_batch_grouped": ([_P, ctypes.c_size_t, _P, _P, _P], ctypes.c_int),
    "pentago_init": ([], ctypes.c_int),
    "pentago_autotune_eval": ([_P, ctypes.c_size_t, _P, _P, _P, _P], ctypes.c_int),
    "pentago_table_counts": ([_P, ctypes.c_uint64, _P, _P], ctypes.c_int),
    "pentago_autotune_sections": ([_P, ctypes.c_size_t, ctypes.c_int, _P, _P, _P, _P], ctypes.c_int),
    "pentago_validate_table": ([_P, ctypes.c_uint64, _P], ctypes.c_int),
    "pentago_set_validate": ([ctypes.c_int], ctypes.c_int),
    "pentago_eval_batch_noalloc": ([_P, ctypes.c_size_t, _P, _P, _P], ctypes.c_int),
    "pentago_serve_create": ([_P, _P], ctypes.c_int),
    "pentago_serve_add_section": ([_P, Section, _P], ctypes.c_int),
    "pentago_serve_submit": ([_P, Board, _P], ctypes.c_int),
    "pentago_serve_poll": ([_P, ctypes.c_uint64, _P], ctypes.c_int),
    "pentago_serve_stats_get": ([_P, _P], ctypes.c_int),
    "pentago_serve_destroy": ([_P], ctypes.c_int),
    "pentago_serve_reset_stats": ([_P], ctypes.c_int),
    "pentago_serve_replay": ([_P, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "pentago_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "pentago_last_error": ([], ctypes.c_char_p),
    "pentago_debug_five": ([Board, ctypes.c_int, _P], ctypes.c_int),
    "pentago_debug_rmax": ([_P, _P], ctypes.c_int),
    "pentago_debug_shift": ([_P, ctypes.c_int, ctypes.c_int, _P], ctypes.c_int),
    "pentago_debug_canon": ([ctypes.c_int, _P, _P], ctypes.c_int),
    "pentago_debug_sym": ([_P, ctypes.c_int, _P, _P], ctypes.c_int),
    "pentago_debug_sym_pattern": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P],
                                  ctypes.c_int),
    "pentago_debug_swap3": ([_P, ctypes.c_int, _P], ctypes.c_int),
}


def lib():
    """Load libpentago.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpentago.so is not built: run paper_1404_0743_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.argtypes = args
                f.restype = res
        _lib = L
    return _lib


def _strerror(code):
    try:
        return lib().pentago_strerror(code).decode()
    except Exception:
        return "error"


def _check(code, func):
    if code != 0:
        raise PentagoError(code, func, lib().pentago_last_error().decode())
    return code


def section(counts):
    """counts ((b0,w0),(b1,w1),(b2,w2),(b3,w3)) -> Section."""
    s = Section()
    for j, (b, w) in enumerate(counts):
        s.black[j], s.white[j] = b, w
    return s


def board(codes):
    b = Board()
    for j in range(4):
        b.q[j] = int(codes[j])
    return b


def boards_to_codes(boards):
    """(n, 36) uint8 cell arrays -> (n, 4) uint16 quadrant codes."""
    boards = np.asarray(boards, dtype=np.int64).reshape(-1, 6, 6)
    codes = np.zeros((len(boards), 4), np.uint16)
    for j in range(4):
        r0, c0 = 3 * (j // 2), 3 * (j % 2)
        q = boards[:, r0:r0 + 3, c0:c0 + 3].reshape(-1, 9)
        codes[:, j] = (q * (3 ** np.arange(9))).sum(axis=1)
    return codes


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------- layout

def pentago_section_shape(counts):
    shape = (ctypes.c_uint32 * 4)()
    entries = ctypes.c_uint64()
    positions = ctypes.c_uint64()
    _check(lib().pentago_section_shape(section(counts), shape, ctypes.byref(entries),
                                       ctypes.byref(positions)), "pentago_section_shape")
    return tuple(shape), entries.value, positions.value


def pentago_section_offset(counts, idx):
    i = (ctypes.c_uint32 * 4)(*[int(x) for x in idx])
    off = ctypes.c_uint64()
    _check(lib().pentago_section_offset(section(counts), i, ctypes.byref(off)),
           "pentago_section_offset")
    return off.value


def pentago_section_board(counts, idx):
    i = (ctypes.c_uint32 * 4)(*[int(x) for x in idx])
    b = Board()
    _check(lib().pentago_section_board(section(counts), i, ctypes.byref(b)), "pentago_section_board")
    return tuple(b.q)


def pentago_child_section(counts, j):
    c = Section()
    _check(lib().pentago_child_section(section(counts), j, ctypes.byref(c)), "pentago_child_section")
    return tuple((c.black[k], c.white[k]) for k in range(4))


# ---------------------------------------------------------------- board symmetries

def _counts_of(sec):
    return tuple((sec.black[k], sec.white[k]) for k in range(4))


def pentago_section_image(counts, sym):
    """Counts of the image section under board symmetry sym (0..7)."""
    c = Section()
    _check(lib().pentago_section_image(section(counts), int(sym), ctypes.byref(c)), "pentago_section_image")
    return _counts_of(c)


def pentago_section_standardize(counts):
    """(representative counts, sym) with pentago_section_image(rep, sym) == counts."""
    c = Section()
    sym = ctypes.c_int()
    _check(lib().pentago_section_standardize(section(counts), ctypes.byref(c), ctypes.byref(sym)),
           "pentago_section_standardize")
    return _counts_of(c), sym.value


def pentago_section_transform(counts, table, sym, out, stream=None):
    """out (device, entries x 64 B) = the table of pentago_section_image(counts, sym)."""
    _check(lib().pentago_section_transform(section(counts), _dev_ptr(table), int(sym), _dev_ptr(out),
                                           _stream(stream)), "pentago_section_transform")


# ---------------------------------------------------------------- sweep

def pentago_solve_section(counts, children, out, stream=None):
    """children: 4 device tensors (or None); out: device tensor of entries x 64 B."""
    ch = (ctypes.c_void_p * 4)(*[None if c is None else c.data_ptr() for c in children])
    for c in children:
        if c is not None:
            _dev_ptr(c)
    _check(lib().pentago_solve_section(section(counts), ch, _dev_ptr(out), _stream(stream)),
           "pentago_solve_section")


def pentago_solve_section_d4(counts, reps, out, stream=None):
    """reps: 4 device tensors holding the tables of the children's
    representatives (pentago_section_standardize), or None."""
    ch = (ctypes.c_void_p * 4)(*[None if c is None else _dev_ptr(c) for c in reps])
    _check(lib().pentago_solve_section_d4(section(counts), ch, _dev_ptr(out), _stream(stream)),
           "pentago_solve_section_d4")


def pentago_autotune_section(counts, children, out, stream=None):
    """Time the tile shapes of this section geometry, remember the fastest;
    returns ({"lines", "threads", "order"}, best ms).  out holds the sweep's
    result afterwards."""
    ch = (ctypes.c_void_p * 4)(*[None if c is None else c.data_ptr() for c in children])
    shape = TileShape()
    ms = ctypes.c_float()
    _check(lib().pentago_autotune_section(section(counts), ch, _dev_ptr(out), _stream(stream),
                                          ctypes.byref(shape), ctypes.byref(ms)),
           "pentago_autotune_section")
    return {"lines": shape.lines, "threads": shape.threads, "order": shape.order}, ms.value


def pentago_solve_section_shape(counts, children, out, lines, threads, order=0, stream=None):
    """The sweep with an explicit tile shape."""
    ch = (ctypes.c_void_p * 4)(*[None if c is None else c.data_ptr() for c in children])
    shape = TileShape(int(lines), int(threads), int(order))
    _check(lib().pentago_solve_section_shape(section(counts), ch, _dev_ptr(out), _stream(stream),
                                             ctypes.byref(shape)),
           "pentago_solve_section_shape")


def _job_array(jobs):
    arr = (SectionJob * len(jobs))()
    for k, (counts, children, out) in enumerate(jobs):
        arr[k].section = section(counts)
        for j in range(4):
            arr[k].child[j] = None if children[j] is None else children[j].data_ptr()
        arr[k].out = out.data_ptr()
    return arr


def pentago_solve_sections(jobs, stream=None):
    """jobs: list of (counts, children (4 tensors or None), out tensor)."""
    arr = _job_array(jobs)
    _check(lib().pentago_solve_sections(arr, len(jobs), _stream(stream)), "pentago_solve_sections")


def pentago_autotune_sections(jobs, reps=False, stream=None):
    """Time the batched sweep's tile shapes (threads per tile, tile LDS cap)
    on these jobs, keep the fastest for their stone count; returns (cap in
    bytes, threads, best ms)."""
    arr = _job_array(jobs)
    cap, nt, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_float()
    _check(lib().pentago_autotune_sections(arr, len(jobs), 1 if reps else 0, _stream(stream), ctypes.byref(cap),
                                           ctypes.byref(nt), ctypes.byref(ms)), "pentago_autotune_sections")
    return cap.value, nt.value, ms.value


def pentago_solve_sections_d4(jobs, stream=None):
    """jobs: list of (counts, tables of the children's representatives (4
    tensors or None), out tensor)."""
    arr = _job_array(jobs)
    _check(lib().pentago_solve_sections_d4(arr, len(jobs), _stream(stream)), "pentago_solve_sections_d4")


def pentago_slice_sections(stones):
    """The D4-minimal sections of a slice, in lexicographic order of counts."""
    n = ctypes.c_size_t()
    _check(lib().pentago_slice_sections(int(stones), None, 0, ctypes.byref(n)), "pentago_slice_sections")
    arr = (Section * max(1, n.value))()
    _check(lib().pentago_slice_sections(int(stones), arr, n.value, ctypes.byref(n)), "pentago_slice_sections")
    return [_counts_of(arr[k]) for k in range(n.value)]


class SweepPlan:
    """pentago_plan_*: one layer's job table kept on the device (reps=True:
    the children are the representatives' tables, pentago_plan_create_d4)."""

    def __init__(self, jobs, reps=False):
        self._keep = jobs
        h = ctypes.c_void_p()
        f = lib().pentago_plan_create_d4 if reps else lib().pentago_plan_create
        _check(f(_job_array(jobs), len(jobs), ctypes.byref(h)),
               "pentago_plan_create" + ("_d4" if reps else ""))
        self.h = h

    def launch(self, stream=None, graph=False):
        f = lib().pentago_plan_launch_graph if graph else lib().pentago_plan_launch
        _check(f(self.h, _stream(stream)), "pentago_plan_launch" + ("_graph" if graph else ""))

    def info(self):
        t, g, l = ctypes.c_longlong(), ctypes.c_int(), ctypes.c_int()
        _check(lib().pentago_plan_info(self.h, ctypes.byref(t), ctypes.byref(g), ctypes.byref(l)),
               "pentago_plan_info")
        return {"tiles": t.value, "grid": g.value, "lds_bytes": l.value}

    def close(self):
        if self.h:
            lib().pentago_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- endgame

def pentago_eval_deep(codes, out, stream=None):
    """One board (4 quadrant codes) solved from scratch; out: device tensor
    of 8 int64 (64 B)."""
    _check(lib().pentago_eval_deep(board(codes), _dev_ptr(out), _stream(stream)), "pentago_eval_deep")


def pentago_eval_deep_parity(codes, parity, out, stream=None):
    """pentago_eval_deep for the rotations of one parity of sum g_i (32 B
    records per node); the other parity's bits of out are zero."""
    _check(lib().pentago_eval_deep_parity(board(codes), int(parity), _dev_ptr(out), _stream(stream)),
           "pentago_eval_deep_parity")


def pentago_eval_batch(boards, out, status=None, stream=None, grouped=False):
    """boards: device tensor (n, 4) int16/uint16 codes (or n x 8 bytes); out:
    device tensor with n x 64 bytes; status: optional device int32 tensor."""
    n = boards.numel() * boards.element_size() // 8
    f = lib().pentago_eval_batch_grouped if grouped else lib().pentago_eval_batch
    _check(f(_dev_ptr(boards), n, _dev_ptr(out), _dev_ptr(status), _stream(stream)),
           "pentago_eval_batch" + ("_grouped" if grouped else ""))


def pentago_autotune_eval(boards, out, stream=None):
    """Time the endgame classes' workgroup sizes on these boards, keep the
    fastest; returns ((threads of class 0, of class 1), best ms)."""
    n = boards.numel() * boards.element_size() // 8
    th = (ctypes.c_int * 2)()
    ms = ctypes.c_float()
    _check(lib().pentago_autotune_eval(_dev_ptr(boards), n, _dev_ptr(out), _stream(stream), th,
                                       ctypes.byref(ms)), "pentago_autotune_eval")
    return (th[0], th[1]), ms.value


def pentago_table_counts(table, out, stream=None):
    """out (device, 4 int64): wins, ties, losses over every (entry,
    rotation) pair of the table, and its invalid entries (stream-ordered)."""
    n = table.numel() * table.element_size() // 64
    _check(lib().pentago_table_counts(_dev_ptr(table), n, _dev_ptr(out), _stream(stream)),
           "pentago_table_counts")


def pentago_validate_table(table, stream=None):
    """Raises PentagoError (EINVAL) if an entry's win set is not inside its
    not-lose set; synchronises the stream."""
    n = table.numel() * table.element_size() // 64
    _check(lib().pentago_validate_table(_dev_ptr(table), n, _stream(stream)), "pentago_validate_table")


def pentago_set_validate(on):
    """Debug-validate mode: the sweeps check their child tables first."""
    _check(lib().pentago_set_validate(1 if on else 0), "pentago_set_validate")


def pentago_init():
    """Upload the tables and resolve the allocation-free call's scratch on the
    current device."""
    _check(lib().pentago_init(), "pentago_init")


def pentago_eval_batch_noalloc(boards, out, status=None, stream=None):
    """pentago_eval_batch with its scratch in the library's fixed device
    array (no allocation); at most 2^20 boards; pentago_init() first."""
    n = boards.numel() * boards.element_size() // 8
    _check(lib().pentago_eval_batch_noalloc(_dev_ptr(boards), n, _dev_ptr(out), _dev_ptr(status),
                                            _stream(stream)), "pentago_eval_batch_noalloc")


# ---------------------------------------------------------------- serving

class Server:
    """pentago_serve_*: create, add resident sections, submit, poll, stats."""

    def __init__(self, memory_budget=1 << 30, max_inflight=4096, max_batch=1024, streams=2):
        cfg = ServeConfig(memory_budget, max_inflight, max_batch, streams)
        h = ctypes.c_void_p()
        _check(lib().pentago_serve_create(ctypes.byref(cfg), ctypes.byref(h)), "pentago_serve_create")
        self.h = h
        self._keep = []

    def add_section(self, counts, table):
        _dev_ptr(table)
        self._keep.append(table)
        _check(lib().pentago_serve_add_section(self.h, section(counts), ctypes.c_void_p(table.data_ptr())),
               "pentago_serve_add_section")

    def submit(self, codes):
        t = ctypes.c_uint64()
        rc = lib().pentago_serve_submit(self.h, board(codes), ctypes.byref(t))
        if rc == EAGAIN:
            return None
        _check(rc, "pentago_serve_submit")
        return t.value

    def poll(self, ticket):
        out = (ctypes.c_uint64 * 8)()
        rc = lib().pentago_serve_poll(self.h, ticket, out)
        if rc == EAGAIN:
            return None
        _check(rc, "pentago_serve_poll")
        return np.array(out, dtype=np.uint64)

    def stats(self):
        s = ServeStats()
        _check(lib().pentago_serve_stats_get(self.h, ctypes.byref(s)), "pentago_serve_stats_get")
        return {k: getattr(s, k) for k, _ in ServeStats._fields_}

    def reset_stats(self):
        _check(lib().pentago_serve_reset_stats(self.h), "pentago_serve_reset_stats")

    def replay(self, codes, arrival_s):
        """Open-loop replay of (n, 4) quadrant codes at the given arrival
        times (seconds); returns (n, 8) uint64 results."""
        codes = np.ascontiguousarray(codes, dtype=np.uint16).reshape(-1, 4)
        t = np.ascontiguousarray(arrival_s, dtype=np.float64)
        out = np.zeros((len(codes), 8), np.uint64)
        _check(lib().pentago_serve_replay(self.h, codes.ctypes.data_as(ctypes.c_void_p),
                                          t.ctypes.data_as(ctypes.c_void_p), len(codes),
                                          out.ctypes.data_as(ctypes.c_void_p)), "pentago_serve_replay")
        return out

    def close(self):
        if self.h:
            _check(lib().pentago_serve_destroy(self.h), "pentago_serve_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- host self-checks

def _set(words):
    s = Set256()
    for i in range(4):
        s.w[i] = int(words[i])
    return s


def pentago_debug_five(codes, color):
    out = Set256()
    _check(lib().pentago_debug_five(board(codes), color, ctypes.byref(out)), "pentago_debug_five")
    return np.array(out.w, dtype=np.uint64)


def pentago_debug_rmax(words):
    src, out = _set(words), Set256()
    _check(lib().pentago_debug_rmax(ctypes.byref(src), ctypes.byref(out)), "pentago_debug_rmax")
    return np.array(out.w, dtype=np.uint64)


def pentago_debug_shift(words, d, k):
    src, out = _set(words), Set256()
    _check(lib().pentago_debug_shift(ctypes.byref(src), d, k, ctypes.byref(out)),
           "pentago_debug_shift")
    return np.array(out.w, dtype=np.uint64)


def pentago_debug_swap3(words, d):
    src, out = _set(words), Set256()
    _check(lib().pentago_debug_swap3(ctypes.byref(src), d, ctypes.byref(out)), "pentago_debug_swap3")
    return np.array(out.w, dtype=np.uint64)


def pentago_debug_sym(words, sym, h):
    """words: 4 u64 (bit g in word g >> 6); h: turns of the 4 image quadrants."""
    src, out = _set(words), Set256()
    hh = (ctypes.c_int * 4)(*[int(x) for x in h])
    _check(lib().pentago_debug_sym(ctypes.byref(src), int(sym), hh, ctypes.byref(out)), "pentago_debug_sym")
    return np.array(out.w, dtype=np.uint64)


def pentago_debug_sym_pattern(sym, black, white, index):
    src = ctypes.c_int()
    h = ctypes.c_int()
    _check(lib().pentago_debug_sym_pattern(int(sym), int(black), int(white), int(index), ctypes.byref(src),
                                           ctypes.byref(h)), "pentago_debug_sym_pattern")
    return src.value, h.value


def pentago_debug_canon(code):
    i, k = ctypes.c_int(), ctypes.c_int()
    _check(lib().pentago_debug_canon(code, ctypes.byref(i), ctypes.byref(k)), "pentago_debug_canon")
    return i.value, k.value
