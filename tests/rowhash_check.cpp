// Host check of the row hash lookup (paper_1411_4942_amd/csrc/rowhash.hpp):
// rowhash_contains must agree with std::binary_search on every query, and
// (built with AddressSanitizer) never read outside a table of exactly
// 2 * slots + kHashPad entries, the size graph preparation allocates.
//
// The table here is built on the host from the layout rule alone (row a owns
// entries [2 off[a], 2 off[a+1]); key b sits at the first empty entry at or
// after its home, wrapping inside the row), not by the GPU build.  The pad
// entries after the last row hold queried keys, so a lookup that let a
// window read past its row count them would answer wrongly.
// Usage: rowhash_check <seed> <slots> <queries>
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../paper_1411_4942_amd/csrc/rowhash.hpp"

int main(int argc, char **argv)
{
    const uint64_t seed = argc > 1 ? strtoull(argv[1], nullptr, 10) : 1;
    const int64_t slots = argc > 2 ? strtoll(argv[2], nullptr, 10) : 100000;
    const int64_t queries = argc > 3 ? strtoll(argv[3], nullptr, 10) : 200000;
    std::mt19937_64 rng(seed);

    // rows with heavy-tailed lengths (empty rows and single slots included),
    // one of them long
    std::vector<int64_t> off{0};
    while (off.back() < slots) {
        int64_t d;
        const uint64_t r = rng() % 100;
        if (off.size() == 3)
            d = slots / 2;
        else if (r < 20)
            d = (int64_t)(rng() % 3);
        else if (r < 60)
            d = (int64_t)(rng() % 16);
        else if (r < 90)
            d = (int64_t)(rng() % 300);
        else
            d = (int64_t)(rng() % 5000);
        // every other row at most a quarter of the slots, so that small
        // tables still hold several rows
        if (off.size() != 3) d = std::min<int64_t>(d, std::max<int64_t>(slots / 4, 1));
        d = std::min<int64_t>(d, slots - off.back());
        off.push_back(off.back() + d);
    }
    const int64_t rows = (int64_t)off.size() - 1;
    // ascending distinct columns per row over a small id range, so that
    // neighbouring rows share keys (a window straddling two rows sees keys
    // of the other row that the query asks for)
    std::vector<uint32_t> col((size_t)std::max<int64_t>(slots, 1));
    for (int64_t r = 0; r < rows; ++r) {
        uint32_t v = (uint32_t)(rng() % 8);
        for (int64_t p = off[r]; p < off[r + 1]; ++p) {
            col[p] = v;
            v += 1 + (uint32_t)(rng() % 3);
        }
    }

    // exactly the size preparation allocates; 16-byte aligned like a device
    // allocation (the windows are 16-byte loads)
    const int64_t entries = 2 * slots + pm::kHashPad;
    void *mem = nullptr;
    if (posix_memalign(&mem, 16, sizeof(uint32_t) * entries) != 0) return 2;
    uint32_t *H = (uint32_t *)mem;
    for (int64_t i = 0; i < 2 * slots; ++i) H[i] = pm::kHashEmpty;
    for (int64_t i = 2 * slots; i < entries; ++i) H[i] = (uint32_t)(i % 8);  // queried keys, not empty
    for (int64_t r = 0; r < rows; ++r) {
        const int64_t d = off[r + 1] - off[r], base = 2 * off[r];
        for (int64_t p = off[r]; p < off[r + 1]; ++p) {
            int64_t q = pm::hash_home(col[p], (uint32_t)(2 * d));
            while (H[base + q] != pm::kHashEmpty) q = (q + 1) % (2 * d);
            H[base + q] = col[p];
        }
    }

    int64_t mismatches = 0, hits = 0;
    for (int64_t i = 0; i < queries; ++i) {
        // rows weighted towards the last ones (the window at the table's end)
        const int64_t r = (i % 5 == 0) ? rows - 1 - (int64_t)(rng() % std::min<int64_t>(rows, 4))
                                       : (int64_t)(rng() % rows);
        const int64_t lo = off[r], d = off[r + 1] - off[r];
        uint32_t key;
        const uint64_t kind = rng() % 4;
        if (kind == 0 && d > 0)
            key = col[lo + (int64_t)(rng() % d)];  // a member
        else if (kind == 1 && r + 1 < rows && off[r + 2] > off[r + 1])
            key = col[off[r + 1] + (int64_t)(rng() % (off[r + 2] - off[r + 1]))];  // the next row's
        else if (kind == 2)
            key = (uint32_t)(rng() % 8);  // the pad's values
        else
            key = (uint32_t)(rng() % (d > 0 ? col[lo + d - 1] + 4 : 16));
        const bool want = std::binary_search(col.begin() + lo, col.begin() + lo + d, key);
        const bool got = pm::rowhash_contains(H, (uint32_t)lo, (uint32_t)d, key);
        hits += want;
        if (got != want) {
            if (mismatches < 10)
                printf("mismatch: row %lld (d=%lld) key %u want %d got %d\n", (long long)r, (long long)d, key,
                       (int)want, (int)got);
            ++mismatches;
        }
    }
    printf("rows=%lld slots=%lld queries=%lld hits=%lld mismatches=%lld\n", (long long)rows, (long long)slots,
           (long long)queries, (long long)hits, (long long)mismatches);
    free(mem);
    return mismatches == 0 ? 0 : 1;
}
