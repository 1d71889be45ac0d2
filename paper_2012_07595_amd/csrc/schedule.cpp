// Work schedules of the tensor-times-block kernels (host logic).
#include "schedule.h"

#include <algorithm>

namespace bks {

void build_schedule(const std::vector<int64_t> &segptr, int E, std::vector<Item> &items,
                    std::vector<Fixup> &fix, int64_t &nslots) {
    const int64_t nseg = (int64_t)segptr.size() - 1;
    const int64_t CH = std::max<int64_t>((int64_t)E * kHeavySteps, 2048);
    items.clear();
    fix.clear();
    nslots = 0;
    int64_t s = 0;
    while (s < nseg) {
        int64_t len = segptr[s + 1] - segptr[s];
        if (len > kLightMax) {
            int64_t nch = (len + CH - 1) / CH;
            if (nch == 1) {
                items.push_back({(int32_t)s, -1, segptr[s], segptr[s + 1], -1, 0});
            } else {
                fix.push_back({(int32_t)s, (int32_t)nslots, (int32_t)nch, 0});
                for (int64_t c = 0; c < nch; ++c) {
                    int64_t b = segptr[s] + c * CH, e = std::min(segptr[s + 1], b + CH);
                    items.push_back({(int32_t)s, -1, b, e, (int32_t)(nslots + c), 0});
                }
                nslots += nch;
            }
            ++s;
        } else {
            int64_t s0 = s;
            while (s < nseg && s - s0 < E && segptr[s + 1] - segptr[s] <= kLightMax) ++s;
            items.push_back({(int32_t)s0, (int32_t)s, 0, 0, -1, 0});
        }
    }
}

void build_group_schedule(const std::vector<int64_t> &segptr, std::vector<Item> &items,
                          std::vector<Fixup> &fix, int64_t &nslots) {
    const int64_t nseg = (int64_t)segptr.size() - 1;
    items.clear();
    fix.clear();
    nslots = 0;
    // smallest power-of-two group that gives each lane at most kGroupLPE entries
    auto group_of = [](int64_t len) {
        int L = 1;
        while (L < 64 && (int64_t)L * kGroupLPE < len) L <<= 1;
        return L;
    };
    int64_t s = 0;
    while (s < nseg) {
        const int64_t len = segptr[s + 1] - segptr[s];
        if (len > (int64_t)64 * kGroupLPE) {
            const int64_t nch = (len + kGroupChunk - 1) / kGroupChunk;
            if (nch == 1) {
                items.push_back({(int32_t)s, -1, segptr[s], segptr[s + 1], -1, 64});
            } else {
                fix.push_back({(int32_t)s, (int32_t)nslots, (int32_t)nch, 0});
                for (int64_t c = 0; c < nch; ++c) {
                    const int64_t b = segptr[s] + len * c / nch, e = segptr[s] + len * (c + 1) / nch;
                    items.push_back({(int32_t)s, -1, b, e, (int32_t)(nslots + c), 64});
                }
                nslots += nch;
            }
            ++s;
            continue;
        }
        // a run of segments that all fit one group width L, 64 / L of them
        const int64_t s0 = s;
        int L = group_of(len);
        ++s;
        while (s < nseg) {
            const int64_t l2 = segptr[s + 1] - segptr[s];
            if (l2 > (int64_t)64 * kGroupLPE) break;
            const int L2 = std::max(L, group_of(l2));
            if ((s - s0 + 1) * L2 > 64) break;
            L = L2;
            ++s;
        }
        items.push_back({(int32_t)s0, (int32_t)s, 0, 0, -1, L});
    }
}

void build_wide_schedule(const std::vector<int64_t> &segptr, int CW, std::vector<Item> &items,
                         std::vector<Fixup> &fix, int64_t &nslots) {
    const int64_t nseg = (int64_t)segptr.size() - 1;
    items.clear();
    fix.clear();
    for (int64_t s = 0; s < nseg; ++s) {
        const int64_t len = segptr[s + 1] - segptr[s];
        // equal chunks: no short remainder chunk that costs a whole partial
        const int64_t nch = len == 0 ? 0 : std::max<int64_t>(1, (len + CW / 2) / CW);
        fix.push_back({(int32_t)s, (int32_t)items.size(), (int32_t)nch, 0});
        for (int64_t c = 0; c < nch; ++c) {
            const int64_t b = segptr[s] + len * c / nch, e = segptr[s] + len * (c + 1) / nch;
            items.push_back({(int32_t)s, -1, b, e, (int32_t)items.size(), 0});
        }
    }
    nslots = (int64_t)items.size();
}

void build_fix_tree(std::vector<Fixup> &fx, int64_t &nslots,
                    std::vector<std::vector<Fixup>> &levels) {
    levels.clear();
    while (true) {
        bool deep = false;
        for (const Fixup &f : fx) deep = deep || f.nslots > kFixFan;
        if (!deep) break;
        std::vector<Fixup> lv, next;
        for (const Fixup &f : fx) {
            if (f.nslots <= kFixFan) {
                next.push_back(f);
                continue;
            }
            const int32_t ng = (f.nslots + kFixFan - 1) / kFixFan;
            for (int32_t g = 0; g < ng; ++g)
                lv.push_back({(int32_t)(nslots + g), f.first_slot + g * kFixFan,
                              std::min<int32_t>(kFixFan, f.nslots - g * kFixFan), 0});
            next.push_back({f.seg, (int32_t)nslots, ng, 0});
            nslots += ng;
        }
        levels.push_back(std::move(lv));
        fx.swap(next);
    }
}

}  // namespace bks
