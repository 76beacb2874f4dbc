"""Writes tests/golden/deep_minimax.tab: the rotation-abstracted tables
(Section III: a win bit and a not-lose bit for each of the 256 quadrant
rotation states) of seeded positions with 11, 12 and 13 empty cells, solved
by the oracle's minimax over the Section II rules (O2).  These are the deep
positions of Section VIII, solved from scratch; the file pins the deep
solver beyond the reach of the per-test oracle runs.

Only the oracle computes values here; the boards come from the seeded
random-play generator (no solver arithmetic in it).  Takes about 15 minutes on
8 cores.

  python tests/golden/make_deep_tables.py
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_1404_0743_amd import inputs as I  # noqa: E402

SEED = 1404074390
EMPTIES = (11, 12, 13)
PER = 3


def main():
    boards = []
    for e in EMPTIES:
        boards.append(I.random_play_boards(PER, 36 - e, 36 - e, seed=SEED + e))
    boards = np.concatenate(boards)
    t0 = time.perf_counter()
    tables = O.minimax_tables(boards, nthreads=len(boards))
    dt = time.perf_counter() - t0
    path = os.path.join(HERE, "deep_minimax.tab")
    with open(path, "w") as f:
        f.write("# Deep positions solved from scratch by minimax over the rules (Section II;\n"
                "# Section VIII solves positions outside the database this way).\n"
                "# Boards: seeded random legal play, seed %d + empty cells, %d per count.\n"
                "# Written by tests/golden/make_deep_tables.py (oracle only), %.0f s.\n"
                "# Columns: 36 cells (0 empty, 1 black, 2 white; cell 6r+c), then the win\n"
                "# words 0..3 and the not-lose words 0..3 as hex (bit g = g0+4g1+16g2+64g3\n"
                "# of word g>>6, g_j counter-clockwise turns of quadrant j).\n" % (SEED, PER, dt))
        for b, t in zip(boards, tables):
            f.write("".join(str(int(x)) for x in b) + " " + " ".join("%016x" % int(w) for w in t) + "\n")
    print("wrote %s (%d boards, %.0f s)" % (path, len(boards), dt))


if __name__ == "__main__":
    main()
