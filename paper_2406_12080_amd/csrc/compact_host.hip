// Host side of the hierarchy compaction (Sec. 5.2, "Compacting the
// Hierarchy"): the tree that the keep flags of hgs_compact_mark leave.  Every
// kept node's parent becomes its nearest kept ancestor (so a node may get
// more than eight children); the new order is breadth-first, root first, the
// children of a node contiguous and in their old order.  No GPU work.
#include <cstring>
#include <vector>

#include "hgs.h"

extern "C" hgs_status hgs_compact_rebuild(const int32_t *parent, const int32_t *child_count, const uint8_t *keep,
                                          int64_t n, int32_t *order, int32_t *new_parent, int32_t *new_child_begin,
                                          int32_t *new_child_count, int64_t *n_out)
{
    if (!parent || !child_count || !keep || !order || !new_parent || !new_child_begin || !new_child_count ||
        !n_out || n <= 0 || n >= (int64_t)0x7FFFFFFF)
        return HGS_ERR_INVALID_ARG;
    if (parent[0] != -1 || !keep[0]) return HGS_ERR_INVALID_ARG;
    // nearest kept proper ancestor and depth in the new tree, in one pass:
    // parents precede their children
    std::vector<int32_t> anc((size_t)n, -1), depth((size_t)n, 0);
    int32_t max_depth = 0;
    for (int64_t i = 1; i < n; ++i) {
        const int32_t p = parent[i];
        if (p < 0 || p >= i || child_count[i] < 0) return HGS_ERR_INVALID_ARG;
        if (child_count[i] == 0 && !keep[i]) return HGS_ERR_INVALID_ARG;  // leaves stay
        anc[i] = keep[p] ? p : anc[p];
        if (keep[i]) {
            depth[i] = depth[anc[i]] + 1;
            if (depth[i] > max_depth) max_depth = depth[i];
        }
    }
    // kept nodes by level (counting sort, old order kept within a level)
    std::vector<int64_t> level_start((size_t)max_depth + 2, 0);
    for (int64_t i = 0; i < n; ++i)
        if (keep[i]) ++level_start[(size_t)depth[i] + 1];
    for (int32_t d = 0; d <= max_depth; ++d) level_start[(size_t)d + 1] += level_start[(size_t)d];
    const int64_t m = level_start[(size_t)max_depth + 1];
    std::vector<int32_t> by_level((size_t)m);
    {
        std::vector<int64_t> fill(level_start.begin(), level_start.end() - 1);
        for (int64_t i = 0; i < n; ++i)
            if (keep[i]) by_level[(size_t)fill[(size_t)depth[i]]++] = (int32_t)i;
    }
    // within a level, group by the parent's new position (counting sort over
    // the previous level's positions, old order kept inside a group)
    std::vector<int32_t> newidx((size_t)n, -1);
    order[0] = 0;
    newidx[0] = 0;
    for (int32_t d = 1; d <= max_depth; ++d) {
        const int64_t a = level_start[(size_t)d], b = level_start[(size_t)d + 1];
        const int64_t pa = level_start[(size_t)d - 1], pb = a;  // the parents' new positions
        std::vector<int64_t> cnt((size_t)(pb - pa) + 1, 0);
        for (int64_t k = a; k < b; ++k) ++cnt[(size_t)(newidx[(size_t)anc[(size_t)by_level[(size_t)k]]] - pa) + 1];
        for (size_t q = 1; q < cnt.size(); ++q) cnt[q] += cnt[q - 1];
        for (int64_t k = a; k < b; ++k) {
            const int32_t i = by_level[(size_t)k];
            const int64_t pos = a + cnt[(size_t)(newidx[(size_t)anc[(size_t)i]] - pa)]++;
            order[pos] = i;
            newidx[(size_t)i] = (int32_t)pos;
        }
    }
    std::memset(new_child_count, 0, sizeof(int32_t) * (size_t)m);
    std::memset(new_child_begin, 0, sizeof(int32_t) * (size_t)m);
    new_parent[0] = -1;
    for (int64_t k = 1; k < m; ++k) {
        const int32_t p = newidx[(size_t)anc[(size_t)order[k]]];
        new_parent[k] = p;
        if (new_child_count[p]++ == 0) new_child_begin[p] = (int32_t)k;
    }
    *n_out = m;
    return HGS_OK;
}
