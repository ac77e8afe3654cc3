// First-fit device-memory sub-allocator with a byte budget.
#include <algorithm>

#include "rmb_common.h"

namespace rmb {

static constexpr size_t kAlign = 256;
static constexpr size_t kMinBlock = size_t(256) << 20;  // 256 MiB

static size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

Arena::~Arena() {
    for (auto &b : blocks_) (void)hipFree(b.base);
}

void *Arena::alloc(size_t bytes) {
    bytes = round_up(std::max<size_t>(bytes, 1), kAlign);
    for (auto &b : blocks_) {
        for (size_t k = 0; k < b.segs.size(); ++k) {
            Seg &s = b.segs[k];
            if (s.used || s.size < bytes) continue;
            if (s.size > bytes) {
                Seg rest{s.off + bytes, s.size - bytes, false};
                s.size = bytes;
                b.segs.insert(b.segs.begin() + k + 1, rest);
            }
            b.segs[k].used = true;
            in_use_ += bytes;
            return b.base + b.segs[k].off;
        }
    }
    // new block; when the budget is reached, give completely free blocks
    // back first (they may be too small for this request)
    size_t want = std::max(bytes, kMinBlock);
    if (reserved_ + want > budget_) want = bytes;
    if (reserved_ + want > budget_) {
        release_free_blocks();
        if (reserved_ + want > budget_) return nullptr;
    }
    void *p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess || p == nullptr) {
        (void)hipGetLastError();
        return nullptr;
    }
    reserved_ += want;
    Block b{(char *)p, want, {}};
    b.segs.push_back(Seg{0, bytes, true});
    if (want > bytes) b.segs.push_back(Seg{bytes, want - bytes, false});
    blocks_.push_back(std::move(b));
    in_use_ += bytes;
    return p;
}

void Arena::release_free_blocks() {
    std::vector<Block> keep;
    for (auto &b : blocks_) {
        if (b.segs.size() == 1 && !b.segs[0].used) {
            (void)hipFree(b.base);
            reserved_ -= b.size;
        } else {
            keep.push_back(std::move(b));
        }
    }
    blocks_ = std::move(keep);
}

void Arena::free(void *p) {
    if (!p) return;
    for (auto &b : blocks_) {
        if ((char *)p < b.base || (char *)p >= b.base + b.size) continue;
        size_t off = (char *)p - b.base;
        for (size_t k = 0; k < b.segs.size(); ++k) {
            if (b.segs[k].off != off || !b.segs[k].used) continue;
            b.segs[k].used = false;
            in_use_ -= b.segs[k].size;
            // coalesce with neighbours
            if (k + 1 < b.segs.size() && !b.segs[k + 1].used) {
                b.segs[k].size += b.segs[k + 1].size;
                b.segs.erase(b.segs.begin() + k + 1);
            }
            if (k > 0 && !b.segs[k - 1].used) {
                b.segs[k - 1].size += b.segs[k].size;
                b.segs.erase(b.segs.begin() + k);
            }
            return;
        }
    }
}

}  // namespace rmb
