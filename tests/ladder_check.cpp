// Host check of the row search index (paper_1411_4942_amd/csrc/ladder.hpp):
// ladder_contains must agree with std::binary_search on every query, and
// (built with AddressSanitizer) never read outside the padded buffers that
// graph preparation allocates.  Usage: ladder_check <seed> <slots> <queries>
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../paper_1411_4942_amd/csrc/ladder.hpp"

int main(int argc, char **argv)
{
    const uint64_t seed = argc > 1 ? strtoull(argv[1], nullptr, 10) : 1;
    const int64_t slots = argc > 2 ? strtoll(argv[2], nullptr, 10) : 100000;
    const int64_t queries = argc > 3 ? strtoll(argv[3], nullptr, 10) : 200000;
    std::mt19937_64 rng(seed);

    // rows with heavy-tailed lengths, one of them very long
    std::vector<int64_t> off{0};
    while (off.back() < slots) {
        int64_t d;
        const uint64_t r = rng() % 100;
        if (off.size() == 3)
            d = slots / 2;
        else if (r < 50)
            d = (int64_t)(rng() % 8);
        else if (r < 90)
            d = (int64_t)(rng() % 200);
        else
            d = (int64_t)(rng() % 5000);
        d = std::min<int64_t>(d, slots - off.back());
        off.push_back(off.back() + d);
    }
    // padded exactly like graph preparation: whole lines plus one line
    const int64_t ssp = (slots + 31) / 32 * 32 + 32;
    uint32_t *col = (uint32_t *)aligned_alloc(128, sizeof(uint32_t) * ssp);
    for (size_t r = 0; r + 1 < off.size(); ++r) {
        uint32_t v = (uint32_t)(rng() % 16);
        for (int64_t p = off[r]; p < off[r + 1]; ++p) {
            col[p] = v;
            v += 1 + (uint32_t)(rng() % 5);
        }
    }
    const int top = pm::ladder_top_for(slots);
    uint64_t lofs[pm::kLadderMax] = {0}, total = 0;
    for (int l = 1; l <= top; ++l) {
        lofs[l] = total;
        total += (pm::ladder_count(slots, l) + 31) / 32 * 32;
    }
    uint32_t *lad = (uint32_t *)aligned_alloc(128, sizeof(uint32_t) * (total + 32));
    pm::Ladder L;
    L.top = top;
    L.lvl[0] = col;
    for (int l = 1; l < pm::kLadderMax; ++l) L.lvl[l] = l <= top ? lad + lofs[l] : nullptr;
    for (int l = 1; l <= top; ++l) {
        const uint32_t *prev = L.lvl[l - 1];
        uint32_t *next = lad + lofs[l];
        for (uint64_t i = 0; i < pm::ladder_count(slots, l); ++i) next[i] = prev[i * 32];
    }

    int64_t bad = 0, hits = 0;
    const size_t rows = off.size() - 1;
    for (int64_t q = 0; q < queries; ++q) {
        const size_t r = (q % 7 == 0 && rows > 2) ? 2 : (size_t)(rng() % rows);  // often the long row
        const int64_t lo = off[r], hi = off[r + 1];
        uint32_t key;
        if (hi > lo && rng() % 2)
            key = col[lo + (int64_t)(rng() % (uint64_t)(hi - lo))];  // present
        else
            key = (uint32_t)(rng() % (uint64_t)(hi > lo ? col[hi - 1] + 20 : 50));
        const bool want = std::binary_search(col + lo, col + hi, key);
        const bool got = pm::ladder_contains(L, (uint32_t)lo, (uint32_t)hi, key);
        hits += want;
        if (want != got) {
            if (bad < 10) fprintf(stderr, "mismatch row %zu [%ld,%ld) key %u want %d got %d\n", r, (long)lo, (long)hi, key, want, got);
            ++bad;
        }
    }
    printf("slots=%ld top=%d rows=%zu queries=%ld present=%ld mismatches=%ld\n", (long)slots, top, rows,
           (long)queries, (long)hits, (long)bad);
    free(col);
    free(lad);
    return bad ? 1 : 0;
}
