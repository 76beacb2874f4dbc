"""Plain CPU oracle for the pentago retrograde sweep -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  The product path (``paper_1404_0743_amd``)
never imports it, and it imports nothing from the product path.

The arithmetic lives in ``pentago_oracle.c`` (plain C, see its header for the
conventions).  This module only compiles it with gcc and marshals arguments.

Oracle functions and what they follow (Irving, arXiv:1404.0743):
  five, turn, apply        -- rules of Section I, f_c of Section II, L of Section III
  value, minimax_tables    -- O2: the v_c / h_c recurrence of Section II, memoised
  section_*                -- Section IV layout (sections, rotation-minimal quadrant
                              orderings, 8^4 blocks) and O4: the Section II
                              recurrence per entry on concrete boards, children read
                              from the (n+1)-stone child sections.
  sym_*, section_transform -- the board symmetries (D4 of Section III) acting on
                              sections and on their tables, bit by bit on concrete
                              boards (Section IV computes only D4-minimal sections).
Parity status: pinned (see tests/test_oracle_*.py); nothing here is unpinned.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pentago_oracle.c")
_LIB = os.path.join(_HERE, "_pentago_oracle.so")

BLACK, WHITE = 1, 2


def build(force=False):
    """Compile the oracle with gcc (always recompiles when force is set)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               "-pthread", "-Wall", "-Wno-unused-function", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.po_init.restype = ctypes.c_int
        L.po_five.argtypes = [P, ctypes.c_int]
        L.po_turn.argtypes = [P, ctypes.c_int, ctypes.c_int]
        L.po_apply.argtypes = [P, ctypes.c_int, P]
        L.po_lines.argtypes = [P]
        L.po_mover.argtypes = [P]
        L.po_value.argtypes = [P]
        L.po_minimax_tables.argtypes = [P, ctypes.c_long, P, ctypes.c_int]
        L.po_class_size.argtypes = [ctypes.c_int, ctypes.c_int]
        L.po_class_code.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.po_code_turn.argtypes = [ctypes.c_int, ctypes.c_int]
        L.po_canon.argtypes = [ctypes.c_int, P]
        L.po_section_entries.argtypes = [P]
        L.po_section_entries.restype = ctypes.c_long
        L.po_section_offset.argtypes = [P, P]
        L.po_section_offset.restype = ctypes.c_long
        L.po_section_board.argtypes = [P, P, P]
        L.po_section_solve.argtypes = [P, P, P, ctypes.c_long, P, ctypes.c_int]
        L.po_section_all_indices.argtypes = [P, P]
        L.po_section_all_indices.restype = ctypes.c_long
        L.po_sym_cells.argtypes = [ctypes.c_int, P]
        L.po_sym_quadrants.argtypes = [ctypes.c_int, P]
        L.po_sym_counts.argtypes = [P, ctypes.c_int, P]
        L.po_section_transform.argtypes = [P, P, ctypes.c_int, P, ctypes.c_long, P, ctypes.c_int]
        L.po_init()
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _board(b):
    b = np.ascontiguousarray(b, dtype=np.uint8)
    assert b.shape == (36,)
    return b


def default_threads():
    return max(1, os.cpu_count() or 1)


# ---------------------------------------------------------------- rules

def five(board, color):
    b = _board(board)
    return lib().po_five(_ptr(b), int(color))


def turn(board, quadrant, turns):
    b = _board(board).copy()
    lib().po_turn(_ptr(b), int(quadrant), int(turns))
    return b


def apply(board, g):
    b = _board(board)
    out = np.zeros(36, np.uint8)
    lib().po_apply(_ptr(b), int(g), _ptr(out))
    return out


def lines():
    out = np.zeros((32, 5), np.int32)
    n = lib().po_lines(_ptr(out))
    return out[:n]


def mover(board):
    return lib().po_mover(_ptr(_board(board)))


def value(board):
    """v_c(s) for the side to move (Section II), by minimax."""
    v = lib().po_value(_ptr(_board(board)))
    if v == -2:
        raise ValueError("invalid board counts")
    return v


def minimax_tables(boards, nthreads=None):
    """(n, 8) uint64 tables: win words then not-lose words, by minimax."""
    boards = np.ascontiguousarray(boards, dtype=np.uint8).reshape(-1, 36)
    out = np.zeros((len(boards), 8), np.uint64)
    rc = lib().po_minimax_tables(_ptr(boards), len(boards), _ptr(out),
                                 nthreads or default_threads())
    if rc:
        raise ValueError("invalid board counts")
    return out


# ---------------------------------------------------------------- quadrants & sections

def class_size(b, w):
    return lib().po_class_size(int(b), int(w))


def class_codes(b, w):
    L = lib()
    return np.array([L.po_class_code(b, w, i) for i in range(L.po_class_size(b, w))], np.int64)


def code_turn(code, turns):
    return lib().po_code_turn(int(code), int(turns))


def canon(code):
    k = ctypes.c_int(0)
    m = lib().po_canon(int(code), ctypes.byref(k))
    return m, k.value


def _counts(counts):
    """counts: ((b0,w0),(b1,w1),(b2,w2),(b3,w3)) -> int32[8] black then white."""
    c = np.zeros(8, np.int32)
    for j, (b, w) in enumerate(counts):
        c[j], c[4 + j] = b, w
    return c


def section_shape(counts):
    return tuple(class_size(b, w) for b, w in counts)


def section_entries(counts):
    n = lib().po_section_entries(_ptr(_counts(counts)))
    if n < 0:
        raise ValueError("invalid section")
    return n


def section_offset(counts, idx):
    i = np.ascontiguousarray(idx, dtype=np.int32)
    off = lib().po_section_offset(_ptr(_counts(counts)), _ptr(i))
    if off < 0:
        raise ValueError("invalid section or index")
    return off


def section_board(counts, idx):
    i = np.ascontiguousarray(idx, dtype=np.int32)
    out = np.zeros(36, np.uint8)
    if lib().po_section_board(_ptr(_counts(counts)), _ptr(i), _ptr(out)):
        raise ValueError("invalid section or index")
    return out


def section_all_indices(counts):
    """All entry indices, row k holding the entry stored at blocked offset k."""
    n = section_entries(counts)
    out = np.zeros((n, 4), np.int32)
    lib().po_section_all_indices(_ptr(_counts(counts)), _ptr(out))
    return out


def child_counts(counts, quadrant):
    """Counts of the child section: the side to move gains a stone in `quadrant`."""
    sb = sum(b for b, _ in counts)
    sw = sum(w for _, w in counts)
    black_moves = sb == sw
    out = [list(x) for x in counts]
    out[quadrant][0 if black_moves else 1] += 1
    return tuple(tuple(x) for x in out)


def section_solve(counts, children, idx=None, nthreads=None):
    """O4.  children: list of 4 host tables ((entries, 8) uint64) or None.
    idx: (n, 4) int32 entry indices, or None for the whole section, in which
    case the result is in blocked-layout order."""
    if idx is None:
        idx = section_all_indices(counts)
    idx = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, 4)
    keep = []
    ptrs = (ctypes.c_void_p * 4)()
    for j in range(4):
        t = children[j] if children is not None else None
        if t is None:
            ptrs[j] = None
        else:
            t = np.ascontiguousarray(t, dtype=np.uint64)
            keep.append(t)
            ptrs[j] = t.ctypes.data
    out = np.zeros((len(idx), 8), np.uint64)
    rc = lib().po_section_solve(_ptr(_counts(counts)), ptrs, _ptr(idx), len(idx), _ptr(out),
                                nthreads or default_threads())
    if rc:
        raise ValueError("section solve failed (%d)" % rc)
    return out


# ------------------------------------------------------------- board symmetries

def sym_cells(sym):
    """Cell map of board symmetry sym = r + 4*f (mirror left-right if f, then
    r counter-clockwise quarter turns): the stone on cell c moves to out[c]."""
    out = np.zeros(36, np.int32)
    if lib().po_sym_cells(int(sym), _ptr(out)):
        raise ValueError("bad symmetry")
    return out


def sym_quadrants(sym):
    out = np.zeros(4, np.int32)
    if lib().po_sym_quadrants(int(sym), _ptr(out)):
        raise ValueError("bad symmetry")
    return tuple(int(x) for x in out)


def sym_counts(counts, sym):
    """Counts of the image section under board symmetry sym."""
    out = np.zeros(8, np.int32)
    if lib().po_sym_counts(_ptr(_counts(counts)), int(sym), _ptr(out)):
        raise ValueError("invalid section or symmetry")
    return tuple((int(out[j]), int(out[4 + j])) for j in range(4))


def section_transform(counts, table, sym, idx=None, nthreads=None):
    """Table of the image section sym(counts) from the whole table of
    `counts` (blocked order), entry by entry and bit by bit.  idx: (n, 4)
    indices of the image section, or None for all of it (blocked order)."""
    dst = sym_counts(counts, sym)
    if idx is None:
        idx = section_all_indices(dst)
    idx = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, 4)
    src = np.ascontiguousarray(table, dtype=np.uint64)
    if src.shape != (section_entries(counts), 8):
        raise ValueError("source table has the wrong shape")
    out = np.zeros((len(idx), 8), np.uint64)
    rc = lib().po_section_transform(_ptr(_counts(counts)), _ptr(src), int(sym), _ptr(idx), len(idx),
                                    _ptr(out), nthreads or default_threads())
    if rc:
        raise ValueError("section transform failed (%d)" % rc)
    return out


# ---------------------------------------------------------------- table helpers

def table_bits(t):
    """(…, 8) uint64 -> (…, 2, 256) bool: [win, notlose] per g."""
    t = np.asarray(t, dtype=np.uint64)
    bits = np.unpackbits(t.view(np.uint8).reshape(t.shape[:-1] + (8, 8)), axis=-1,
                         bitorder="little")
    return bits.reshape(t.shape[:-1] + (2, 256)).astype(bool)


def table_values(t):
    """(…, 8) uint64 -> (…, 256) int8 values in {-1, 0, 1}."""
    b = table_bits(t)
    return (b[..., 0, :].astype(np.int8) + b[..., 1, :].astype(np.int8) - 1)
