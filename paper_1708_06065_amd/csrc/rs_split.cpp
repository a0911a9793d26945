// The library's own classical CF splitting: the Ruge-Stueben first pass
// without a second pass (the splitting the paper uses, Sec. 4).  It is a
// greedy sequential algorithm, so it runs on the host between the device
// strength kernel and the device neighbourhood kernels.
//
// Measure lambda_i = number of points that strongly depend on i.  Points
// with no strong connection in either direction are F.  Repeatedly the
// undecided point with the largest measure (smallest index among equals)
// becomes C; the undecided points depending on it become F and every
// undecided point those new F-points depend on gains one; the undecided
// points the new C-point depends on lose one.  When the largest remaining
// measure is zero the rest become F.
//
// The arg-max is a binary max-heap of (measure, index) with lazy deletion:
// an entry is live only if it matches the point's current measure and the
// point is still undecided.
#include <cstdint>
#include <queue>
#include <utility>
#include <vector>

namespace lair {

void rs_first_pass(int64_t n, const int32_t *rp, const int32_t *cj,
                   const uint8_t *sm, int8_t *cf) {
    std::vector<int64_t> tp((size_t)n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
            if (sm[p]) tp[(size_t)cj[p] + 1]++;
    for (int64_t i = 0; i < n; ++i) tp[i + 1] += tp[i];
    std::vector<int32_t> tj((size_t)tp[n]);
    {
        std::vector<int64_t> fill(tp.begin(), tp.end() - 1);
        for (int64_t i = 0; i < n; ++i)
            for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
                if (sm[p]) tj[(size_t)fill[cj[p]]++] = (int32_t)i;
    }
    enum : int8_t { UNDECIDED = -1, FPT = 0, CPT = 1 };
    std::vector<int8_t> st((size_t)n, UNDECIDED);
    std::vector<int64_t> lam((size_t)n, 0);
    // heap ordering: larger measure first, then smaller index
    using Key = std::pair<int64_t, int64_t>;   // (measure, -index)
    std::priority_queue<Key> heap;
    for (int64_t i = 0; i < n; ++i) {
        bool has_out = false;
        for (int32_t p = rp[i]; p < rp[i + 1] && !has_out; ++p) has_out = sm[p] != 0;
        lam[i] = tp[i + 1] - tp[i];
        if (!has_out && lam[i] == 0) {
            st[i] = FPT;
        } else {
            heap.push(Key(lam[i], -i));
        }
    }
    auto bump = [&](int64_t k, int64_t d) {
        lam[k] += d;
        heap.push(Key(lam[k], -k));
    };
    while (!heap.empty()) {
        Key top = heap.top();
        heap.pop();
        int64_t i = -top.second;
        if (st[i] != UNDECIDED || lam[i] != top.first) continue;   // stale
        if (top.first == 0) {
            for (int64_t k = 0; k < n; ++k)
                if (st[k] == UNDECIDED) st[k] = FPT;
            break;
        }
        st[i] = CPT;
        for (int64_t q = tp[i]; q < tp[i + 1]; ++q) {
            int32_t j = tj[q];
            if (st[j] != UNDECIDED) continue;
            st[j] = FPT;
            for (int32_t p = rp[j]; p < rp[j + 1]; ++p) {
                int32_t k = cj[p];
                if (sm[p] && st[k] == UNDECIDED) bump(k, +1);
            }
        }
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
            int32_t j = cj[p];
            if (sm[p] && st[j] == UNDECIDED) bump(j, -1);
        }
    }
    for (int64_t i = 0; i < n; ++i) cf[i] = (st[i] == CPT) ? 1 : 0;
}

}  // namespace lair
