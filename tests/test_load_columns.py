"""Host-side check of the uint8 kernels' load addresses (no GPU).

The kernels take their per-lane load columns from csrc/load_columns.hpp.
This test compiles that same header with g++ and enumerates every lane of
every tile the single-image launch (four tiles side by side per wave, idle
groups included) and the batched launch can produce, for many widths: every
block a lane loads must hold at least one byte of the row, so that no load
of the aligned-row path reaches past the row's last aligned block.
"""
import pathlib
import shutil
import subprocess

import pytest

CSRC = pathlib.Path(__file__).resolve().parents[1] / "paper_2305_00515_amd" / "csrc"

PROGRAM = r"""
#include <cstdio>
#include <initializer_list>
#include "load_columns.hpp"
using namespace s4x5;
static int bad = 0;
static void check(int W, int ppl, int xo, int lane16, const char *what) {
    const LoadCols c = load_columns(xo, lane16, W, ppl);
    const bool ok_blk = c.ldx % ppl == 0 && (int)c.ldx < W;             // block holds column ldx < W
    const bool ok_hx = c.hx % 4 == 0 && (int)c.hx < W;                  // dword holds column hx < W
    if (!ok_blk || !ok_hx) {
        if (bad < 10) std::printf("BAD %s W=%d ppl=%d xo=%d lane16=%d ldx=%u hx=%u\n", what, W, ppl, xo, lane16, c.ldx, c.hx);
        ++bad;
    }
}
int main() {
    int widths[700], n = 0;
    for (int w = 1; w <= 600; ++w) widths[n++] = w;
    const int big[] = {767, 768, 769, 1000, 1023, 1024, 1025, 1920, 2047, 2048, 3840, 4095, 4096, 4099, 8192, 16383, 16384};
    for (int w : big) widths[n++] = w;
    for (int i = 0; i < n; ++i) {
        const int W = widths[i];
        for (int valid = 0; valid < 2; ++valid) {
            const int Wo = valid ? W - 4 : W;
            if (Wo < 1) continue;
            for (int ppl : {8, 16}) {
                const int tw = 16 * ppl, ntx = (Wo + tw - 1) / tw;
                // single image: strips of four tiles side by side, idle groups included
                for (int tx = 0; tx < ((ntx + 3) / 4) * 4; ++tx)
                    for (int l = 0; l < 16; ++l) check(W, ppl, tx * tw + l * ppl, l, "single");
                // batched: tiles of the image only
                for (int tx = 0; tx < ntx; ++tx)
                    for (int l = 0; l < 16; ++l) check(W, ppl, tx * tw + l * ppl, l, "batched");
            }
        }
    }
    std::printf(bad ? "FAIL %d\n" : "ok\n", bad);
    return bad != 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_every_load_holds_a_byte_of_the_row(tmp_path):
    src = tmp_path / "cols.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "cols"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", str(CSRC), str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout


FOLD_PROGRAM = r"""
#include <cstdio>
#include "load_columns.hpp"
using namespace s4x5;
// the definition, written out: step by one pixel, bouncing off both edges
static int walk(int i, int n) {
    if (n == 1) return 0;
    int pos = 0, dir = i >= 0 ? 1 : -1;
    for (int k = 0; k != (i >= 0 ? i : -i); ++k) {
        if (pos + dir < 0 || pos + dir > n - 1) dir = -dir;
        pos += dir;
    }
    return pos;
}
int main() {
    int bad = 0;
    for (int n = 1; n <= 70; ++n)
        for (int i = -3 * n - 5; i <= 4 * n + 5; ++i) {
            const int r = reflect101(i, n);
            if (r < 0 || r >= n || r != walk(i, n)) {
                if (bad < 10) std::printf("BAD n=%d i=%d got %d want %d\n", n, i, r, walk(i, n));
                ++bad;
            }
        }
    std::printf(bad ? "FAIL %d\n" : "ok\n", bad);
    return bad != 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_reflect101_index_map(tmp_path):
    """The kernels' reflect-101 map stays inside [0, n-1] for every index and
    equals a walk that bounces off both edges without repeating them."""
    src = tmp_path / "fold.cpp"
    src.write_text(FOLD_PROGRAM)
    exe = tmp_path / "fold"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", str(CSRC), str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout
