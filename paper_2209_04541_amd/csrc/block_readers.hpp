// Which in-flight counting windows still read a resident block.
//
// The streamer deals windows (groups of tasks whose blocks are resident
// together) round-robin over several compute streams.  Windows on one stream
// finish in order, but windows on different streams may finish in any order,
// so before a block's device range is reused, every stream's last window
// that read the block must have finished -- the last window overall is not
// enough: an earlier, heavier window on another stream may still be reading
// it.  This keeps, per block and per stream, the last window that read the
// block since it was loaded.
//
// Host-only code (no HIP types), so the bookkeeping can be checked on the
// CPU.
#pragma once

#include <cstdint>
#include <vector>

namespace pgabb {

class BlockReaders {
  public:
    BlockReaders(int32_t nblocks, int nstreams)
        : nstreams_(nstreams), last_(static_cast<size_t>(nblocks) * nstreams, -1) {}

    // Window `window` on compute stream `stream` reads `block`.  Windows are
    // numbered in issue order, so on one stream a later call has a larger
    // window.
    void read(int32_t block, int stream, int32_t window) {
        last_[static_cast<size_t>(block) * nstreams_ + stream] = window;
    }

    // Before the block's memory is reused: calls wait(w) for the last window
    // w on each stream that read the block (waiting for w covers the earlier
    // windows on its stream) and forgets them.
    template <class Wait>
    void release(int32_t block, Wait &&wait) {
        int32_t *row = &last_[static_cast<size_t>(block) * nstreams_];
        for (int s = 0; s < nstreams_; ++s) {
            if (row[s] >= 0) wait(row[s]);
            row[s] = -1;
        }
    }

    // Forget every reader (after all streams were synchronized).
    void clear() { last_.assign(last_.size(), -1); }

  private:
    int nstreams_;
    std::vector<int32_t> last_;
};

}  // namespace pgabb
