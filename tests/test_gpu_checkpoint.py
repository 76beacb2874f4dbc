"""Kill and resume: the 35-stone sections a layer of 34-stone sections needs
are solved, written to disk and dropped; a fresh start reads them back and
solves the 34-stone layer, which must be the same bytes as the layer solved
straight from the tables in memory (the paper restarted its last slices
from the slices it had written out, Section VI)."""
import sys

import pytest
import torch

from paper_1404_0743_amd import checkpoint as C
from paper_1404_0743_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1404_0743_amd import pentago
    pentago.lib()
    return pentago


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_resume_layer_from_saved_children(P, tmp_path):
    secs = I.pick_layer_sections(34, count=12, lo=1e3, hi=3e6, seed=9134)
    children = {}
    for s in secs:
        for j in range(4):
            if sum(s[j]) < 9:
                children[P.pentago_child_section(s, j)] = None
    log("layer 34:", len(secs), "sections,", len(children), "children")
    for c in children:
        t = torch.empty((P.pentago_section_shape(c)[1], 8), dtype=torch.int64, device="cuda")
        P.pentago_solve_section(c, [None] * 4, t)
        children[c] = t
    torch.cuda.synchronize()

    def layer(tables):
        outs = []
        for s in secs:
            ch = [tables[P.pentago_child_section(s, j)] if sum(s[j]) < 9 else None for j in range(4)]
            o = torch.empty((P.pentago_section_shape(s)[1], 8), dtype=torch.int64, device="cuda")
            outs.append((s, ch, o))
        P.pentago_solve_sections(outs)
        torch.cuda.synchronize()
        return [o for _, _, o in outs]

    direct = layer(children)
    for c, t in children.items():
        C.save_table(C.table_path(str(tmp_path), c), c, t)
    del children
    torch.cuda.empty_cache()
    # a fresh start: the child layer comes back from disk only
    loaded = {}
    for c in {P.pentago_child_section(s, j) for s in secs for j in range(4) if sum(s[j]) < 9}:
        counts, t = C.load_table(C.table_path(str(tmp_path), c), device="cuda")
        assert counts == c
        loaded[c] = t
    resumed = layer(loaded)
    for s, a, b in zip(secs, direct, resumed):
        assert torch.equal(a, b), s
