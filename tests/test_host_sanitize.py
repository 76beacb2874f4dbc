"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the C oracle (rules, minimax, the section retrograde, the symmetry
transform) built with gcc, and the library's host table builders (quadrant
classes, line structure, symmetry maps, per-pattern lookups, DAG layouts)
built with hipcc, the sanitizers applied to host code only.  Each driver
runs in a subprocess; any report fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")

ORACLE_DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
int po_init(void);
int po_five(const uint8_t *b, int x);
int po_value(const uint8_t *b);
int po_minimax_tables(const uint8_t *boards, long n, uint64_t *out, int nthreads);
long po_section_entries(const int *counts);
long po_section_all_indices(const int *counts, int *idx);
int po_section_solve(const int *counts, const uint64_t *const *child, const int *idx, long n,
                     uint64_t *out, int nthreads);
int po_sym_counts(const int *counts, int sym, int *out);
int po_section_transform(const int *counts, const uint64_t *src, int sym, const int *idx, long n,
                         uint64_t *out, int nthreads);

int main(void)
{
    po_init();
    /* a board with 3 empty cells, 17 black and 16 white stones (valid
       counts, white to move) */
    uint8_t b[36];
    for (int i = 0, k = 0; i < 36; i++) {
        if (i == 3 || i == 17 || i == 30) { b[i] = 0; continue; }
        b[i] = (uint8_t)(k % 2 == 0 ? 1 : 2);
        k++;
    }
    uint64_t t[8];
    if (po_minimax_tables(b, 1, t, 2)) return 2;
    /* a 35-stone section solved whole, then transformed by a reflection */
    const int counts[8] = {9, 0, 4, 5, 0, 9, 4, 4};
    const long n = po_section_entries(counts);
    int *idx = malloc(sizeof(int) * 4 * (size_t)n);
    uint64_t *tab = malloc(sizeof(uint64_t) * 8 * (size_t)n);
    uint64_t *img = malloc(sizeof(uint64_t) * 8 * (size_t)n);
    if (!idx || !tab || !img || po_section_all_indices(counts, idx) != n) return 3;
    if (po_section_solve(counts, NULL, idx, n, tab, 2)) return 4;
    int ic[8];
    if (po_sym_counts(counts, 5, ic)) return 5;
    int *iidx = malloc(sizeof(int) * 4 * (size_t)n);
    if (!iidx || po_section_all_indices(ic, iidx) != n) return 6;
    if (po_section_transform(counts, tab, 5, iidx, n, img, 2)) return 7;
    unsigned long long acc = 0;
    for (long i = 0; i < 8 * n; i++) acc += tab[i] ^ img[i];
    printf("ok %ld %llu\n", n, acc);
    free(idx); free(iidx); free(tab); free(img);
    return 0;
}
"""

HOST_DRIVER = r"""
#include <cstdio>
#include "tables.h"
int main()
{
    const pg::HostTables &H = pg::host_tables();
    unsigned long long acc = H.qinfo.size() + H.symmap.size() + H.syminv.size() + H.pat_lm.size() +
                             H.pat_sel.size() + H.pat_child.size();
    for (int e = 0; e <= 10; e++) acc += pg::dag_layout(e).node.size() + pg::dag_layout(e).edge.size();
    std::printf("ok %llu\n", acc);
    return 0;
}
"""


PLANTED = r"""
#include <stdlib.h>
int main(int argc, char **argv)
{
    int *a = malloc(4 * sizeof(int));
    a[argc + 3] = 1;   /* one past the end */
    int r = a[0];
    free(a);
    return r;
}
"""


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, env=ENV, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-3000:], r.stderr[-6000:])
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("no gcc")
    (tmp_path / "drv.c").write_text(ORACLE_DRIVER)
    _run(["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-pthread", "drv.c", os.path.join(ROOT, "oracle", "pentago_oracle.c"),
          "-o", "drv"], tmp_path)
    out = _run([str(tmp_path / "drv")], tmp_path)
    assert out.startswith("ok ")


def test_host_tables_under_asan_ubsan(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("no hipcc")
    csrc = os.path.join(ROOT, "paper_1404_0743_amd", "csrc")
    (tmp_path / "drv.cpp").write_text(HOST_DRIVER)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    _run([hipcc, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer"] + san +
         ["-I", csrc, "drv.cpp", os.path.join(csrc, "tables.cpp"), "-o", "drv"], tmp_path)
    out = _run([str(tmp_path / "drv")], tmp_path)
    assert out.startswith("ok ")


def test_sanitizer_reports_a_planted_error(tmp_path):
    """The same flags catch a heap overflow (the harness would see it)."""
    if not shutil.which("gcc"):
        pytest.skip("no gcc")
    (tmp_path / "bad.c").write_text(PLANTED)
    _run(["gcc", "-std=c99", "-O0", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "bad.c", "-o", "bad"], tmp_path)
    r = subprocess.run([str(tmp_path / "bad")], cwd=tmp_path, env=ENV, capture_output=True, text=True, timeout=60)
    assert r.returncode == 23 and "heap-buffer-overflow" in r.stderr
