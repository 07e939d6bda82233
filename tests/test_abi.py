"""The C ABI: the built library loads without a GPU, exports every entry
point include/lpa.h declares, and the binding's ctypes layouts match the C
structs.  No compute call is made here."""
import ctypes
import os
import re
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lpa.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lpa_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2301_09125_amd import lpa
    lib = lpa.library()
    names = declared()
    assert set(names) == set(lpa.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", lpa.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (lpa_\w+)", out))
    assert set(names) <= exported


def test_default_options_and_strerror():
    from paper_2301_09125_amd import lpa
    o = lpa.default_options()
    assert o == {"self_weight": 1, "thread_max": 8, "group_max": 32, "wave_max": 128, "wide_max": 512, "merge_max": 512, "frontier": 0,
                 "profile": 0, "modularity": 0, "barrier_timeout_us": 0, "order": 0, "tie": 0,
                 "seed": 0, "reuse_csr": 0}
    lib = lpa.library()
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert lib.lpa_strerror(code)
    assert lib.lpa_strerror(-99) == b"unknown status"


def test_ctypes_layouts_match_c():
    from paper_2301_09125_amd import lpa
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "lpa.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(lpa_csr), sizeof(lpa_options), sizeof(lpa_stats),
         sizeof(lpa_kernel_prof), offsetof(lpa_stats, changed_per_iter), offsetof(lpa_kernel_prof, ms),
         sizeof(lpa_batch_stats), offsetof(lpa_batch_stats, iterations), offsetof(lpa_batch_stats, hist_cap));
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(lpa_mlp), offsetof(lpa_mlp, tau), sizeof(lpa_learned_stats),
         offsetof(lpa_learned_stats, cap), sizeof(lpa_train_options), offsetof(lpa_train_options, recall));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        got = [int(x) for x in subprocess.check_output([exe]).split()]
    want = [ctypes.sizeof(lpa._Csr), ctypes.sizeof(lpa._Options), ctypes.sizeof(lpa._Stats),
            ctypes.sizeof(lpa._KProf), lpa._Stats.changed_per_iter.offset, lpa._KProf.ms.offset,
            ctypes.sizeof(lpa._BatchStats), lpa._BatchStats.iterations.offset, lpa._BatchStats.hist_cap.offset,
            ctypes.sizeof(lpa._Mlp), lpa._Mlp.tau.offset, ctypes.sizeof(lpa._LearnedStats), lpa._LearnedStats.cap.offset,
            ctypes.sizeof(lpa._TrainOpts), lpa._TrainOpts.recall.offset]
    assert got == want


def test_header_documents_each_entry_point():
    text = open(HEADER).read()
    for n in declared():
        i = text.index(n + "(")
        before = text[:i]
        assert before.rstrip().endswith("*/") or "lpa_status" in before[-40:] or "void" in before[-40:] \
            or "const char" in before[-40:], n
