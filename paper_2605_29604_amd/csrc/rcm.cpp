// Reverse Cuthill-McKee ordering (host): a breadth-first numbering that keeps
// neighbours close, so mesh-like graphs get banded adjacency and dense diagonal
// tiles.  Each component starts at an unnumbered vertex of minimum degree (ties:
// smallest id); neighbours are numbered by increasing degree, then id; the final
// order is reversed.  Sequential by nature, so it runs on the host during the build.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "../../include/tcmis.h"

namespace tcmis {

int host_rcm(const int64_t* rp, const int32_t* ci, int64_t n, std::vector<int32_t>& new_id) {
    std::vector<int64_t> deg(n);
    for (int64_t v = 0; v < n; ++v) deg[v] = rp[v + 1] - rp[v];
    auto less = [&](int32_t a, int32_t b) { return deg[a] < deg[b] || (deg[a] == deg[b] && a < b); };
    // the vertices by increasing degree, then id: a counting sort on the degree (stable,
    // so ids stay increasing within a degree)
    int64_t dmax = 0;
    for (int64_t v = 0; v < n; ++v) dmax = std::max(dmax, deg[v]);
    std::vector<int64_t> first(dmax + 2, 0);
    for (int64_t v = 0; v < n; ++v) ++first[deg[v] + 1];
    for (int64_t d = 0; d <= dmax; ++d) first[d + 1] += first[d];
    std::vector<int32_t> by_deg(n);
    for (int64_t v = 0; v < n; ++v) by_deg[first[deg[v]]++] = (int32_t)v;
    std::vector<uint8_t> seen(n, 0);
    std::vector<int32_t> order;
    order.reserve(n);
    std::vector<int32_t> nb;
    size_t start = 0, head = 0;
    while ((int64_t)order.size() < n) {
        if (head == order.size()) {
            while (seen[by_deg[start]]) ++start;
            seen[by_deg[start]] = 1;
            order.push_back(by_deg[start]);
        }
        const int32_t v = order[head++];
        nb.clear();
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
            const int32_t u = ci[e];
            if (!seen[u]) { seen[u] = 1; nb.push_back(u); }
        }
        std::sort(nb.begin(), nb.end(), less);
        order.insert(order.end(), nb.begin(), nb.end());
    }
    std::reverse(order.begin(), order.end());
    new_id.assign(n, 0);
    for (int64_t p = 0; p < n; ++p) new_id[order[p]] = (int32_t)p;
    return MIS_OK;
}

}  // namespace tcmis
