"""Section tables on disk, so that a sweep of several layers can stop after any
layer and resume from the files of the layer above (the paper writes out the
slices it computes and restarted its remaining slices from them, Section VI).

A file is a 128-byte header, then the table's entries x 64 bytes exactly as
they sit in device memory (8^4-blocked order).  The header holds a magic and
a layout version, the section's counts, its shape and number of entries, the
table's win / tie / loss counts over every (entry, rotation) pair (the
per-slice counts of Section VII, a check of the values) and a CRC-32 of the
table bytes.  load_table verifies all of it and raises ValueError on any
mismatch."""
import os
import struct
import zlib

import numpy as np

from . import pentago as P

MAGIC = b"PNTGTBL\0"
VERSION = 1
# magic, version, counts (black 4, white 4), shape (4 x u32), entries,
# win, tie, loss (u64 each), crc32, padding to 128 bytes
_HEAD = struct.Struct("<8sI8B4IQQQQI")
HEADER_BYTES = 128
_CHUNK = 1 << 28


def _host_bytes(table):
    """The table as a C-contiguous uint64 numpy array (copied to the host if
    it lives on the GPU)."""
    if hasattr(table, "is_cuda"):
        table = table.detach()
        if table.is_cuda:
            table = table.cpu()
        table = table.contiguous().numpy()
    return np.ascontiguousarray(table).view(np.uint64).reshape(-1, 8)


def table_counts_host(t):
    """wins, ties, losses over every (entry, rotation) pair of a host table."""
    w, n = t[:, :4], t[:, 4:]
    win = tie = nl = 0
    for a in range(0, len(t), 1 << 20):
        wa, na = w[a:a + (1 << 20)], n[a:a + (1 << 20)]
        win += int(np.bitwise_count(wa).sum())
        tie += int(np.bitwise_count(na & ~wa).sum())
        nl += int(np.bitwise_count(na).sum())
    return win, tie, 256 * len(t) - nl


def _crc(t):
    b = t.view(np.uint8).reshape(-1)
    c = 0
    for a in range(0, len(b), _CHUNK):
        c = zlib.crc32(b[a:a + _CHUNK], c)
    return c & 0xffffffff


def save_table(path, counts, table):
    """Write the table of section `counts` (device tensor or host array,
    entries x 64 bytes) to path, atomically (a temporary file renamed)."""
    shape, entries, _ = P.pentago_section_shape(counts)
    t = _host_bytes(table)
    if len(t) != entries:
        raise ValueError("table has %d entries, section %s has %d" % (len(t), counts, entries))
    win, tie, loss = table_counts_host(t)
    head = _HEAD.pack(MAGIC, VERSION, *[b for b, _ in counts], *[w for _, w in counts], *shape, entries,
                      win, tie, loss, _crc(t))
    tmp = "%s.tmp%d" % (path, os.getpid())
    with open(tmp, "wb") as f:
        f.write(head.ljust(HEADER_BYTES, b"\0"))
        f.write(t.tobytes())
    os.replace(tmp, path)


def load_table(path, device=None):
    """(counts, table) from a file written by save_table: the table as a
    host uint64 array (entries x 8), or as an int64 tensor on `device`.
    Raises ValueError if the header, size, counts or checksum do not match."""
    with open(path, "rb") as f:
        head = f.read(HEADER_BYTES)
        if len(head) != HEADER_BYTES:
            raise ValueError("%s: short header" % path)
        fields = _HEAD.unpack(head[:_HEAD.size])
        magic, version = fields[0], fields[1]
        if magic != MAGIC or version != VERSION:
            raise ValueError("%s: not a section table of layout version %d" % (path, VERSION))
        black, white = fields[2:6], fields[6:10]
        shape, entries = list(fields[10:14]), fields[14]
        win, tie, loss, crc = fields[15:19]
        counts = tuple((int(b), int(w)) for b, w in zip(black, white))
        want_shape, want_entries, _ = P.pentago_section_shape(counts)
        if list(want_shape) != shape or want_entries != entries:
            raise ValueError("%s: shape does not match section %s" % (path, counts))
        t = np.fromfile(f, dtype=np.uint64)
    if t.size != 8 * entries:
        raise ValueError("%s: %d bytes of table, expected %d" % (path, 8 * t.size, 64 * entries))
    t = t.reshape(-1, 8)
    if _crc(t) != crc:
        raise ValueError("%s: checksum mismatch" % path)
    if table_counts_host(t) != (win, tie, loss):
        raise ValueError("%s: win / tie / loss counts do not match" % path)
    if device is None:
        return counts, t
    import torch
    return counts, torch.from_numpy(t.view(np.int64)).to(device)


def table_path(directory, counts):
    """The file name of a section's table in a checkpoint directory."""
    return os.path.join(directory, "s_" + "_".join("%d%d" % bw for bw in counts) + ".tab")
