// Work schedules of the tensor-times-block kernels (host logic, no HIP):
// how the segments of an entry stream (slices, rows or stored pairs) are cut
// into wave-sized items, and how the partial rows of split segments are
// summed back.
#pragma once

#include <cstdint>
#include <vector>

namespace bks {

// One wave-sized unit of work.  Heavy items cover [beg, end) of a single
// long segment; light items cover whole short segments seg .. seg_end-1.
struct Item {
    int32_t seg;
    int32_t seg_end;  // light: one past the last segment; heavy: -1
    int64_t beg, end; // heavy entry range
    int32_t slot;     // heavy split segment: partial slot, else -1
    int32_t pad;      // group schedules: lanes per segment (see build_group_schedule)
};

struct Fixup {
    int32_t seg;
    int32_t first_slot;
    int32_t nslots;
    int32_t pad;
};

// Schedules: heavy items take CH = max(E * kHeavySteps, 2048) entries; light segments
// are at most kLightMax entries long.
constexpr int kHeavySteps = 32;
constexpr int kLightMax = 48;
void build_schedule(const std::vector<int64_t> &segptr, int E, std::vector<Item> &items,
                    std::vector<Fixup> &fix, int64_t &nslots);
// Register-direct narrow products: segments of at most 64 * kGroupLPE
// entries are taken by groups of L lanes (L a power of two, the smallest with
// at most kGroupLPE entries per lane), 64 / L consecutive segments per item
// (light item; `pad` = L, segments seg .. seg_end-1); longer segments are cut
// into ceil(len / kGroupChunk) chunks of equal size (+-1) for one whole wave
// each (heavy item, `pad` = 64), with partial slots and fixups when a segment
// has more than one chunk.  Every segment, empty ones included, is covered.
constexpr int kGroupLPE = 8;
constexpr int64_t kGroupChunk = 2048;
void build_group_schedule(const std::vector<int64_t> &segptr, std::vector<Item> &items,
                          std::vector<Fixup> &fix, int64_t &nslots);
// Wide symmetric products: every nonempty slice of len entries is cut into
// max(1, round(len / CW)) chunks of equal size (+-1 entry), one item each
// (slot = item index), so chunks hold between CW / 2 and 1.5 CW entries
// unless the slice is shorter; fix[s] lists slice s's items (every slice,
// empty ones with nslots = 0).  Cached as order kWideOrder.
constexpr int kWideOrder = 3;
// Group schedules are cached as order kGroupOrder + format (0 slices, 1 pair
// rows, 2 pairs).
constexpr int kGroupOrder = 8;
void build_wide_schedule(const std::vector<int64_t> &segptr, int CW, std::vector<Item> &items,
                         std::vector<Fixup> &fix, int64_t &nslots);
// Fixed-order reduction tree for segments with more than kFixFan partial
// slots: each level's Fixups sum up to kFixFan slots into the new slot named
// by their `seg` field (slots appended after nslots, which grows); levels run
// in order, then `fix` (rewritten to the last level's slots) sums into the
// output rows.
constexpr int kFixFan = 64;
void build_fix_tree(std::vector<Fixup> &fix, int64_t &nslots,
                    std::vector<std::vector<Fixup>> &levels);

}  // namespace bks
