// Edge-list ingest: the undirected simple graph of a list of vertex pairs, as
// CSR, built on the device.  Every pair stands for an undirected edge (both
// directions become slots), self-loops are dropped and repeated pairs merged
// -- the clean-up the paper applies to its input graphs before counting
// (Section 6: direction ignored, duplicates and self-loops removed).
//
//   1. expand: pair (a, b), a != b -> directed entries (a, b) and (b, a);
//      loops -> a sentinel row n that sorts last
//   2. stable radix sort by column, then by row: entries ordered (row, col)
//   3. keep the first of each run of equal entries (not the sentinels);
//      exclusive scan of the keep flags gives each kept entry its slot
//   4. compact the columns; row offsets from where the row changes
#include "graph.hpp"
#include "profile.hpp"
#include "radix.hpp"
#include "scan.hpp"

namespace pm {

pm_status graph_create(const pm_csr_view *csr, uint32_t flags, hipStream_t s, pm_graph **out);

namespace {

enum : uint32_t { ING_RANGE = 1u };

__global__ __launch_bounds__(kBlock) void k_expand(const int32_t *__restrict__ src, const int32_t *__restrict__ dst,
                                                   int64_t E, int64_t n, uint32_t *__restrict__ rows,
                                                   uint32_t *__restrict__ cols, uint32_t *err)
{
    uint32_t e_or = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = src[e], b = dst[e];
        const bool bad = a < 0 || a >= n || b < 0 || b >= n;
        if (bad) e_or |= ING_RANGE;
        if (bad || a == b) {
            rows[2 * e] = rows[2 * e + 1] = (uint32_t)n;
            cols[2 * e] = cols[2 * e + 1] = 0u;
        } else {
            rows[2 * e] = (uint32_t)a;
            cols[2 * e] = (uint32_t)b;
            rows[2 * e + 1] = (uint32_t)b;
            cols[2 * e + 1] = (uint32_t)a;
        }
    }
    if (e_or) atomicOr(err, e_or);
}

// keep flag of sorted entry i: a real row and not equal to entry i-1
struct KeepIn {
    const uint32_t *rows, *cols;
    uint32_t n;
    __device__ __forceinline__ uint32_t operator()(int64_t i) const
    {
        const uint32_t r = rows[i];
        if (r >= n) return 0u;
        return (i == 0 || rows[i - 1] != r || cols[i - 1] != cols[i]) ? 1u : 0u;
    }
};
struct PosOut {
    uint32_t *pos;  // exclusive prefix of the keep flags
    __device__ __forceinline__ void operator()(int64_t i, uint32_t incl, uint32_t x) const { pos[i] = incl - x; }
};

// Compaction and row offsets.  Entry i (and a virtual entry M standing for
// the end) sets off[v] = pos[i] for every row v in (row[i-1], row[i]]: the
// rows it starts and the empty rows before it.
__global__ __launch_bounds__(kBlock) void k_compact(const uint32_t *__restrict__ rows,
                                                    const uint32_t *__restrict__ cols,
                                                    const uint32_t *__restrict__ pos, int64_t M, int64_t n,
                                                    uint32_t total, int64_t *__restrict__ off,
                                                    int32_t *__restrict__ col_out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= M; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i < M ? (int64_t)rows[i] : n;
        const int64_t prev = i > 0 ? (int64_t)rows[i - 1] : -1;
        const uint32_t p = i < M ? pos[i] : total;
        if (i < M && r < n && (i == 0 || prev != r || cols[i - 1] != cols[i])) col_out[p] = (int32_t)cols[i];
        if (r != prev) {
            const int64_t hi = r < n ? r : n;
            for (int64_t v = prev + 1; v <= hi; ++v) off[v] = p;
        }
    }
}

struct IngestOut {
    int64_t slots = 0;
};

// The CSR of the edge list into off[n+1] and col[capacity] (device).
pm_status csr_from_edges_impl(const pm_edge_view *ev, int64_t *off, int32_t *col, int64_t capacity, int64_t *slots_out,
                              hipStream_t s)
{
    const int64_t n = ev->n, E = ev->num_edges;
    Temps tmp(s);
    const int32_t *src = ev->src, *dst = ev->dst;
    if (!ev->on_device && E > 0) {
        int32_t *ds = nullptr, *dd = nullptr;
        PM_TRY(tmp.get(&ds, (size_t)E));
        PM_TRY(tmp.get(&dd, (size_t)E));
        PM_HIP(hipMemcpyAsync(ds, src, sizeof(int32_t) * E, hipMemcpyHostToDevice, s));
        PM_HIP(hipMemcpyAsync(dd, dst, sizeof(int32_t) * E, hipMemcpyHostToDevice, s));
        src = ds;
        dst = dd;
    }
    const int64_t M = 2 * E;
    uint32_t *err = nullptr;
    PM_TRY(tmp.get(&err, 1));
    PM_TRY(fill_async<uint32_t>(err, 0u, 1, s));
    uint32_t *r0 = nullptr, *c0 = nullptr, *r1 = nullptr, *c1 = nullptr, *r2 = nullptr, *c2 = nullptr;
    const size_t mm = (size_t)(M > 0 ? M : 1);
    PM_TRY(tmp.get(&r0, mm));
    PM_TRY(tmp.get(&c0, mm));
    PM_TRY(tmp.get(&r1, mm));
    PM_TRY(tmp.get(&c1, mm));
    PM_TRY(tmp.get(&r2, mm));
    PM_TRY(tmp.get(&c2, mm));
    if (E > 0) {
        ProfScope prof("ingest.expand", s);
        hipLaunchKernelGGL(k_expand, dim3(grid_for(E, kBlock, 1 << 22)), dim3(kBlock), 0, s, src, dst, E, n, r0, c0,
                           err);
        PM_HIP(hipGetLastError());
    }
    uint32_t herr = 0;
    PM_HIP(hipMemcpyAsync(&herr, err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    if (herr & ING_RANGE) {
        set_error("edge list: an endpoint is not a vertex id in [0, n)");
        return PM_EGRAPH;
    }
    // (row, col) order: stable by column, then stable by row
    const int bits = bits_for((uint64_t)n);
    const uint32_t *rows = r0, *cols = c0;
    if (M > 1) {
        char *scr = nullptr;
        PM_TRY(tmp.get(&scr, radix_scratch_bytes(M)));
        uint32_t *kc = nullptr, *vr = nullptr;
        PM_TRY(radix_sort("ingest.sort_col", c0, r0, c1, r1, c2, r2, M, bits, scr, s, &kc, &vr));
        // kc / vr now in (c1, r1) or (c2, r2); sort by row into the other pair and r0 / c0
        uint32_t *ka = (kc == c1) ? c2 : c1, *va = (vr == r1) ? r2 : r1;
        uint32_t *kr = nullptr, *vc = nullptr;
        PM_TRY(radix_sort("ingest.sort_row", vr, kc, ka, va, r0, c0, M, bits, scr, s, &kr, &vc));
        rows = kr;
        cols = vc;
    }
    // keep flags -> slots
    uint32_t *pos = nullptr;
    PM_TRY(tmp.get(&pos, mm));
    uint32_t total = 0;
    if (M > 0) {
        char *scr = nullptr;
        PM_TRY(tmp.get(&scr, ScanScratch<uint32_t>::bytes_for(M, 8)));
        ProfScope prof("ingest.dedup", s);
        PM_TRY((scan_launch<uint32_t, 8>(KeepIn{rows, cols, (uint32_t)n}, PosOut{pos}, M, SumOp<uint32_t>(), 0u, scr,
                                         s)));
        uint32_t last_pos = 0;
        PM_HIP(hipMemcpyAsync(&last_pos, pos + (M - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        // the last entry's own flag: recompute it on the host side of the copy
        uint32_t lr = 0, lc = 0, pr = 0, pc = 0;
        PM_HIP(hipMemcpyAsync(&lr, rows + (M - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        PM_HIP(hipMemcpyAsync(&lc, cols + (M - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        if (M > 1) {
            PM_HIP(hipMemcpyAsync(&pr, rows + (M - 2), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
            PM_HIP(hipMemcpyAsync(&pc, cols + (M - 2), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        }
        PM_HIP(hipStreamSynchronize(s));
        const bool keep_last = lr < (uint32_t)n && (M == 1 || pr != lr || pc != lc);
        total = last_pos + (keep_last ? 1u : 0u);
    }
    if ((int64_t)total > capacity) {
        set_error("edge list: the CSR needs " + std::to_string(total) + " column slots, capacity is " +
                  std::to_string(capacity));
        return PM_EINVAL;
    }
    {
        ProfScope prof("ingest.compact", s);
        hipLaunchKernelGGL(k_compact, dim3(grid_for(M + 1, kBlock, 1 << 22)), dim3(kBlock), 0, s, rows, cols, pos, M,
                           n, total, off, col);
        PM_HIP(hipGetLastError());
    }
    *slots_out = total;
    return PM_OK;
}

pm_status check_edge_view(const pm_edge_view *ev)
{
    if (!ev || ev->n < 0 || ev->n > (int64_t)INT32_MAX - 1 || ev->num_edges < 0 ||
        (ev->num_edges > 0 && (!ev->src || !ev->dst)) || 2 * ev->num_edges >= (int64_t)UINT32_MAX) {
        set_error("edge list: n in [0, 2^31 - 1), 0 <= num_edges < 2^31, src and dst given");
        return PM_EINVAL;
    }
    return PM_OK;
}

}  // namespace

pm_status csr_from_edges(const pm_edge_view *ev, int64_t *off, int32_t *col, int64_t capacity, int64_t *slots_out,
                         hipStream_t s)
{
    PM_TRY(check_edge_view(ev));
    if (!off || !slots_out || capacity < 0 || (capacity > 0 && !col)) {
        set_error("edge list: null output or negative capacity");
        return PM_EINVAL;
    }
    ProfScope prof("ingest_total", s);
    return csr_from_edges_impl(ev, off, col, capacity, slots_out, s);
}

pm_status graph_from_edges(const pm_edge_view *ev, uint32_t flags, hipStream_t s, pm_graph **out)
{
    PM_TRY(check_edge_view(ev));
    if (!out) {
        set_error("edge list: null output");
        return PM_EINVAL;
    }
    *out = nullptr;
    Temps tmp(s);
    int64_t *off = nullptr;
    int32_t *col = nullptr;
    const int64_t cap = 2 * ev->num_edges;
    PM_TRY(tmp.get(&off, (size_t)(ev->n + 1)));
    PM_TRY(tmp.get(&col, (size_t)(cap > 0 ? cap : 1)));
    int64_t slots = 0;
    {
        ProfScope prof("ingest_total", s);
        PM_TRY(csr_from_edges_impl(ev, off, col, cap, &slots, s));
    }
    pm_csr_view v;
    v.n = ev->n;
    v.row_offsets = off;
    v.cols = col;
    v.on_device = 1;
    return graph_create(&v, flags, s, out);
}

}  // namespace pm
