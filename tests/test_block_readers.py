"""CPU check of the streamer's block-reader bookkeeping (csrc/block_readers.hpp).

Windows of tasks are dealt round-robin over several compute streams; a
stream finishes its windows in order, different streams in any order.  Before
a block's device range is reused, every window that read the block since it
was loaded must have finished.  A g++-built driver simulates random window
sequences, random per-stream completion and random evictions, and checks that
after the waits BlockReaders asks for, no reader of the evicted block is still
running.  A negative control checks that waiting only for the block's last
reader (over all streams) does fail under the same model.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2209_04541_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>
#include "block_readers.hpp"

// Model: windows 0..W-1, window w on stream w % S.  done[w] says whether it
// finished.  Streams finish in order: completing w completes every earlier
// window of its stream.
int main(int argc, char **argv) {
    const int naive = argc > 1 && argv[1][0] == 'n';
    int failures = 0;
    for (int trial = 0; trial < 4000; ++trial) {
        std::mt19937 rng(trial);
        const int S = 2 + trial % 3, NB = 6 + trial % 7, W = 40;
        pgabb::BlockReaders br(NB, S);
        std::vector<int> last(NB, -1);                 // naive: last reader overall
        std::vector<std::set<int>> readers(NB);        // ground truth since load
        std::vector<char> done(W, 0);
        auto complete = [&](int w) {                   // what waiting on w guarantees
            for (int x = w; x >= 0; x -= S) done[x] = 1;
        };
        for (int w = 0; w < W; ++w) {
            // some earlier windows finish, in stream order
            for (int k = 0; k < 3; ++k) {
                const int s = rng() % S;
                int first = -1;
                for (int x = s; x < w; x += S)
                    if (!done[x]) { first = x; break; }
                if (first >= 0 && rng() % 2) done[first] = 1;
            }
            // evict a random block, then check none of its readers still runs
            const int v = rng() % NB;
            if (naive) {
                if (last[v] >= 0) complete(last[v]);
                last[v] = -1;
            } else {
                br.release(v, [&](int32_t x) { complete(x); });
            }
            for (int x : readers[v])
                if (!done[x]) { ++failures; break; }
            readers[v].clear();
            // window w reads a few blocks
            const int nr = 1 + rng() % 3;
            for (int q = 0; q < nr; ++q) {
                const int b = rng() % NB;
                readers[b].insert(w);
                last[b] = w;
                br.read(b, w % S, w);
            }
        }
    }
    printf("%d\n", failures);
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("readers")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I" + HDR, str(src), "-o", str(exe)])
    return str(exe)


def test_every_reader_finished_before_reuse(driver):
    out = subprocess.check_output([driver]).decode().strip()
    assert out == "0"


def test_last_reader_alone_is_not_enough(driver):
    """Negative control: the model catches the race of waiting for one window."""
    out = subprocess.check_output([driver, "naive"]).decode().strip()
    assert int(out) > 0
