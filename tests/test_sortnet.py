"""The batched vote's in-register sorting network (csrc/lpa_sortnet.h):
Batcher's odd-even merge sort, restricted to the pairs below D.  Built here
with g++ (the header is plain C++17) and checked by the 0-1 principle on
every 0-1 input of D <= 20 positions (a comparator network sorts every
input iff it sorts every 0-1 input), and against std::sort on random inputs
with many repeats up to D = 32.  Also pins the comparator counts of the
full networks (19, 63 and 191 for 8, 16 and 32 inputs)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2301_09125_amd", "csrc")

DRIVER = r"""
#include "lpa_sortnet.h"
#include <algorithm>
#include <cstdio>
#include <random>
using namespace lpa;
template <int D> int check() {
    constexpr SortNet net = SortNetFor<D>::net;
    for (int c = 0; c < net.n; ++c)
        if (!(net.a[c] < net.b[c] && net.b[c] < D)) { std::printf("D=%d bad pair\n", D); return 1; }
    uint32_t x[D], y[D];
    if (D <= 20) {
        for (uint64_t m = 0; m < (1ull << D); ++m) {
            for (int i = 0; i < D; ++i) x[i] = (uint32_t)(m >> i) & 1u;
            for (int c = 0; c < net.n; ++c) {
                const uint32_t p = x[net.a[c]], q = x[net.b[c]];
                x[net.a[c]] = std::min(p, q);
                x[net.b[c]] = std::max(p, q);
            }
            for (int i = 1; i < D; ++i)
                if (x[i - 1] > x[i]) { std::printf("D=%d fails on 0-1 input %llx\n", D, (unsigned long long)m); return 1; }
        }
    }
    std::mt19937_64 rng(D);
    for (int t = 0; t < 20000; ++t) {
        const uint32_t range = t % 3 == 0 ? 3u : (t % 3 == 1 ? 40u : 0xFFFFFFFFu);
        for (int i = 0; i < D; ++i) y[i] = x[i] = (uint32_t)(rng() % ((uint64_t)range + 1));
        for (int c = 0; c < net.n; ++c) {
            const uint32_t p = x[net.a[c]], q = x[net.b[c]];
            x[net.a[c]] = std::min(p, q);
            x[net.b[c]] = std::max(p, q);
        }
        std::sort(y, y + D);
        for (int i = 0; i < D; ++i)
            if (x[i] != y[i]) { std::printf("D=%d fails on a random input\n", D); return 1; }
    }
    std::printf("D=%d pairs=%d\n", D, net.n);
    return 0;
}
template <int... Ds> int all() { return (check<Ds>() | ...); }
int main() {
    return all<1, 2, 3, 4, 5, 7, 8, 9, 12, 15, 16, 17, 20, 23, 24, 25, 28, 31, 32>();
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_sort_network_sorts(tmp_path):
    src = tmp_path / "sortnet.cpp"
    exe = tmp_path / "sortnet"
    src.write_text(DRIVER)
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    pairs = dict(line.replace("D=", "").split(" pairs=") for line in out.stdout.splitlines())
    # Batcher's odd-even merge sort: 19, 63 and 191 comparators for 8, 16, 32
    assert pairs["8"] == "19" and pairs["16"] == "63" and pairs["32"] == "191"
