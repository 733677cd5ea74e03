"""Host-side check of the dense Tabu kernel's copy of Q (qb_tabu_pos in the
library's internal header, used by the builder kernel on the device): for
every elements-per-thread count, element size and workgroup size it places
each element once within the row pitch, a thread's elements up to 16 bytes
fill the front of one aligned power-of-two slot, and beyond that each
chunk is contiguous and naturally aligned for one vector load.  Compiled with hipcc for the
host only (the header also holds device code); no GPU work."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROG = r"""
#include <cstdio>
#include <vector>
#include "qb_internal.h"
int main() {
    const int opts[] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16};
    int bad = 0;
    for (int tb : {512, 1024})
        for (int esz : {1, 2})
            for (int ept : opts) {
                const int pitch = qb_tabu_pitch(tb, ept, esz);
                const int slot = qb_tabu_slot(ept, esz);
                if (pitch < tb * ept) ++bad;
                std::vector<int> seen(pitch, 0);
                for (int t = 0; t < tb; ++t) {
                    int prev = -2;
                    for (int e = 0; e < ept; ++e) {
                        const int pos = qb_tabu_pos(e, t, ept, esz, tb);
                        if (pos < 0 || pos >= pitch) { ++bad; continue; }
                        ++seen[pos];
                        if (ept * esz <= 16) {
                            // one slot per thread: a power of two of at most
                            // 16 bytes, aligned, holding the elements in order
                            const int sb = slot * esz;
                            if (sb > 16 || (sb & (sb - 1)) != 0 || slot < ept) ++bad;
                            if (pos != t * slot + e) ++bad;
                            continue;
                        }
                        // a new chunk starts where the position is not the next element
                        if (pos != prev + 1) {
                            // the chunk's first element is aligned to the chunk size
                            int sz = 1;
                            while (e + sz < ept && qb_tabu_pos(e + sz, t, ept, esz, tb) == pos + sz) ++sz;
                            if ((pos * esz) % (sz * esz) != 0) ++bad;
                            if (sz * esz > 16 || (sz & (sz - 1)) != 0) ++bad;
                        }
                        prev = pos;
                    }
                }
                int used = 0;
                for (int c : seen) { bad += c > 1; used += c; }
                bad += used != tb * ept;
            }
    std::printf("%d\n", bad);
    return bad != 0;
}
"""


def test_tabu_copy_layout_is_an_aligned_permutation():
    cxx = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(cxx):
        pytest.skip("no hipcc")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "layout.cpp")
        exe = os.path.join(d, "layout")
        open(src, "w").write(PROG)
        subprocess.check_call([cxx, "-x", "hip", "--offload-arch=gfx950", "--cuda-host-only", "-std=c++17", "-O1",
                               "-I" + os.path.join(ROOT, "include"),
                               "-I" + os.path.join(ROOT, "paper_2502_13947_amd", "csrc"), src, "-o", exe])
        out = subprocess.run([exe], capture_output=True, text=True)
        assert out.returncode == 0 and out.stdout.strip() == "0", out.stdout + out.stderr
