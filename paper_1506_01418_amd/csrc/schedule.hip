// Host-side work schedule of one part for the sparse iteration kernel.
//
// The part's blocks are (b, (b + p) mod B).  Every row of W belongs to the
// block of its row piece and every column of H to the block of its column
// piece, and each is one "item" whose gradient is a sum over its entries in
// that block.  Work-groups take items of one block and one side:
//  * items with more than Q * L entries (Q groups per work-group, L entries
//    per group) are cut into n_split shares of one work-group each;
//  * other items get G = 2^k groups, the fewest that leave at most L
//    entries per group, and work-groups pack Q / G such items;
//  * work-groups are placed on the 8 XCDs block by block (a block's rows
//    and columns share an XCD, so the partner rows each side gathers are
//    the ones the other side reads, in that XCD's L2), and dispatch order
//    interleaves the XCD lists because consecutive work-group ids go to
//    consecutive XCDs.
#include <algorithm>
#include <climits>
#include <numeric>
#include <vector>

#include "internal.hpp"

namespace psgld {

namespace {
constexpr int kXcds = 8;

int ceil_log2(int64_t v)
{
    int k = 0;
    while ((int64_t{1} << k) < v) ++k;
    return k;
}

struct Staged {
    WgTask task;
    std::vector<GroupRec> recs;
    int64_t weight;   // larger first within an XCD
};
}  // namespace

void build_part_schedule(const int32_t *pre_r, const int32_t *pre_c, int64_t I, int64_t J,
                         const std::vector<int32_t> &row_piece, const std::vector<int32_t> &col_piece,
                         int32_t B, int32_t p, int lpg, const ScheduleParams &prm, const uint8_t *skip_block,
                         PartSchedule &out)
{
    const int Q = sparse_block_threads() / lpg;
    const int qlog = ceil_log2(Q);
    const int kEntriesPerGroup = std::max(1, prm.entries_per_group);
    const int64_t split_thresh = prm.split_items ? static_cast<int64_t>(Q) * kEntriesPerGroup : INT64_MAX;
    const bool remap = prm.xcd_remap;

    std::vector<std::vector<int32_t>> rows_of(B), cols_of(B);
    for (int64_t i = 0; i < I; ++i) rows_of[row_piece[i]].push_back(static_cast<int32_t>(i));
    for (int64_t j = 0; j < J; ++j) cols_of[((col_piece[j] - p) % B + B) % B].push_back(static_cast<int32_t>(j));

    // block -> XCD: greedy balance of entries + items when there are enough blocks
    std::vector<int> xcd_of(B, 0);
    if (B >= kXcds) {
        std::vector<int64_t> w(B, 0);
        for (int32_t b = 0; b < B; ++b) {
            w[b] = static_cast<int64_t>(rows_of[b].size() + cols_of[b].size());
            for (int32_t i : rows_of[b]) w[b] += pre_r[i + 1] - pre_r[i];
        }
        std::vector<int32_t> order(B);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) { return w[a] > w[c]; });
        std::vector<int64_t> load(kXcds, 0);
        for (int32_t b : order) {
            const int x = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
            xcd_of[b] = x;
            load[x] += w[b];
        }
    }
    std::vector<std::vector<Staged>> lists(kXcds);
    int rr = 0;
    auto place = [&](int32_t b, Staged &&s) {
        const int x = (B >= kXcds && remap) ? xcd_of[b] : (rr++ % kXcds);
        lists[x].push_back(std::move(s));
    };

    out.n_splits = 0;
    for (int32_t b = 0; b < B; ++b) {
        if (skip_block && skip_block[b]) continue;
        for (int side = 0; side < 2; ++side) {
            const std::vector<int32_t> &items = side == 0 ? rows_of[b] : cols_of[b];
            const int32_t *pre = side == 0 ? pre_r : pre_c;
            std::vector<std::pair<int64_t, int32_t>> light;   // (glog2 << 32 | entries, item)
            for (int32_t it : items) {
                const int64_t beg = pre[it], n = pre[it + 1] - pre[it];
                if (n > split_thresh) {
                    const int64_t ns = (n + split_thresh - 1) / split_thresh;
                    const int32_t first = out.n_splits;
                    out.n_splits += static_cast<int32_t>(ns);
                    for (int64_t s = 0; s < ns; ++s) {
                        const int64_t a0 = beg + n * s / ns, a1 = beg + n * (s + 1) / ns;
                        Staged st;
                        st.task = WgTask{static_cast<int16_t>(side), static_cast<int16_t>(qlog), first, static_cast<int32_t>(s),
                                          static_cast<int32_t>(ns)};
                        st.recs.resize(Q);
                        for (int g = 0; g < Q; ++g)
                            st.recs[g] = GroupRec{it, static_cast<int32_t>(a0 + (a1 - a0) * g / Q),
                                                  static_cast<int32_t>(a0 + (a1 - a0) * (g + 1) / Q), g == 0};
                        st.weight = (int64_t{1} << 40) + (a1 - a0);
                        place(b, std::move(st));
                    }
                } else {
                    const int64_t need = (n + kEntriesPerGroup - 1) / kEntriesPerGroup;
                    const int64_t gl = std::min(qlog, ceil_log2(std::max<int64_t>(need, 1)));
                    light.emplace_back((gl << 32) | n, it);
                }
            }
            // by group count, then entry count (similar loop lengths within a wave)
            std::stable_sort(light.begin(), light.end(),
                             [](const std::pair<int64_t, int32_t> &a, const std::pair<int64_t, int32_t> &c) {
                                 return a.first > c.first;
                             });
            size_t pos = 0;
            while (pos < light.size()) {
                const int gl = static_cast<int>(light[pos].first >> 32);
                const int G = 1 << gl, per = Q / G;
                Staged st;
                st.task = WgTask{static_cast<int16_t>(side), static_cast<int16_t>(gl), -1, 0, 0};
                st.recs.assign(Q, GroupRec{-1, 0, 0, 0});
                int64_t max_n = 0;
                for (int k = 0; k < per && pos < light.size() && (light[pos].first >> 32) == gl; ++k, ++pos) {
                    const int32_t it = light[pos].second;
                    const int64_t beg = pre[it], n = pre[it + 1] - pre[it];
                    max_n = std::max(max_n, n);
                    for (int sub = 0; sub < G; ++sub)
                        st.recs[k * G + sub] = GroupRec{it, static_cast<int32_t>(beg + n * sub / G),
                                                        static_cast<int32_t>(beg + n * (sub + 1) / G), sub == 0};
                }
                st.weight = (static_cast<int64_t>(gl) << 32) + max_n;
                place(b, std::move(st));
            }
        }
    }

    // heaviest first within each XCD, then interleave the XCD lists
    size_t longest = 0;
    for (auto &l : lists) {
        std::stable_sort(l.begin(), l.end(), [](const Staged &a, const Staged &c) { return a.weight > c.weight; });
        longest = std::max(longest, l.size());
    }
    out.tasks.clear();
    out.recs.clear();
    for (size_t r = 0; r < longest; ++r)
        for (int x = 0; x < kXcds; ++x) {
            if (r < lists[x].size()) {
                out.tasks.push_back(lists[x][r].task);
                out.recs.insert(out.recs.end(), lists[x][r].recs.begin(), lists[x][r].recs.end());
            } else if (remap && B >= kXcds) {
                out.tasks.push_back(WgTask{0, 0, -1, 0, 0});
                out.recs.insert(out.recs.end(), Q, GroupRec{-1, 0, 0, 0});
            }
        }
}

}  // namespace psgld
