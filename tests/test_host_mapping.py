"""Host logic without a GPU: the workgroup -> supercell order of the particle
and migration kernels is a permutation of the supercells for every grid the
library accepts (a block that missed a supercell would leave its particles
unpushed; two blocks on one supercell would race)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1606_02862_amd", "csrc")

PROGRAM = r'''
#include "pic_internal.hpp"
#include <cstdio>
#include <vector>
int main() {
    int bad = 0, n = 0, zfast = 0;
    for (int ncx = 1; ncx <= 40; ++ncx) for (int ncy = 1; ncy <= 12; ++ncy) for (int ncz = 1; ncz <= 40; ++ncz) {
        const int nsc = ncx * ncy * ncz, nxy = ncx * ncy, per = nsc / 8;
        // the choice pic_init makes
        const int remap = (nsc % 8 != 0) ? 0 : (per % nxy == 0) ? per / nxy : 1;
        zfast += remap > 1;
        std::vector<int> seen(nsc, 0);
        for (int b = 0; b < nsc; ++b) {
            const int sc = pic::sc_of_block(b, nsc, nxy, remap);
            if (sc < 0 || sc >= nsc || seen[sc]++) { ++bad; break; }
        }
        ++n;
    }
    // 128^3 cells in 8x8x4 supercells: each XCD's slab is 4 z-layers walked z fastest,
    // so blocks 0, 8, 16, 24 take the four layers of supercell column (0, 0)
    const int nxy = 16 * 16;
    for (int k = 0; k < 4; ++k)
        if (pic::sc_of_block(8 * k, 16 * 16 * 32, nxy, 4) != k * nxy) ++bad;
    if (pic::sc_of_block(8 * 4, 16 * 16 * 32, nxy, 4) != 1) ++bad;
    if (pic::sc_of_block(1, 16 * 16 * 32, nxy, 4) != 1024) ++bad;
    std::printf("%d %d %d\n", n, zfast, bad);
    return bad != 0;
}
'''


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_block_to_supercell_order_is_a_permutation(tmp_path):
    src = tmp_path / "order.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "order"
    r = subprocess.run(["hipcc", "-O1", f"-I{CSRC}", str(src), "-o", str(exe)],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    n, zfast, bad = map(int, r.stdout.split())
    assert n == 19200 and bad == 0
    assert zfast > 100  # the z-fastest order is exercised, not only the plain slabs
