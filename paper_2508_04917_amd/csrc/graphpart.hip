// Partition labels for a matrix graph without geometry (Section 3: labels
// from a graph partitioner; Section 5.3: parts balanced to one size), as a
// stand-in for METIS: recursive BFS bisection into parts of exactly S
// vertices.  A segment of k parts (k*S vertices, all labelled with its first
// part number b) splits, if k > 1, by a BFS inside the segment from its
// smallest vertex, a second BFS from the reached vertex of largest distance
// (smallest index on ties), and the order (distance, index) with unreached
// vertices last: the first floor(k/2)*S vertices keep label b, the rest take
// b + floor(k/2).  Every segment of one depth is processed at once: the BFS
// levels relax all segments together (edges between segments are ignored),
// and one stable radix sort of (label, distance) keys orders all segments.
// After the last depth, the labels are the part numbers, and the vertices
// are renumbered by a stable sort on the label (Algorithm 3's order).
#include <hipcub/hipcub.hpp>

#include "internal.h"

namespace ddilu {

namespace {

constexpr uint32_t kInf = 0xffffffffu;
constexpr int kT = 256;
constexpr int kLevelBatch = 16;  // BFS levels launched between checks for progress

inline unsigned blocks(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

__global__ void k_gp_fill(int64_t n, int32_t *a, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ void k_gp_fill64(int64_t n, unsigned long long *a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0ull;
}

// smallest vertex of every segment that splits at this depth
__global__ void k_gp_vmin(int64_t n, const int32_t *label, const int32_t *segk, int32_t *src) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t b = label[v];
    // the plain read skips the atomic once a smaller vertex is in (a stale
    // read only costs an atomic that does not change the minimum)
    if (segk[b] > 1 && (int32_t)v < src[b]) atomicMin(&src[b], (int32_t)v);
}

__global__ void k_gp_src(int64_t n, const int32_t *label, const int32_t *segk, const int32_t *src,
                         uint32_t *dist) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t b = label[v];
    dist[v] = (segk[b] > 1 && src[b] == (int32_t)v) ? 0u : kInf;
}

// one BFS level: the vertices at distance d reach their unvisited neighbours
// of the same segment (every writer stores the same d + 1)
__global__ void k_gp_level(int64_t n, const int32_t *ptr, const int32_t *col, const int32_t *label, uint32_t d,
                           uint32_t *dist, int32_t *changed) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n || dist[v] != d) return;
    const int32_t b = label[v];
    bool any = false;
    for (int32_t q = ptr[v]; q < ptr[v + 1]; ++q) {
        const int32_t u = col[q];
        if (label[u] == b && dist[u] == kInf) {
            dist[u] = d + 1;
            any = true;
        }
    }
    if (any) *changed = 1;
}

// reached vertex of largest distance, smallest index on ties, per segment
__global__ void k_gp_far(int64_t n, const int32_t *label, const int32_t *segk, const uint32_t *dist,
                         unsigned long long *far) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n || dist[v] == kInf) return;
    const int32_t b = label[v];
    const unsigned long long key = ((unsigned long long)dist[v] << 32) | (unsigned long long)(~(uint32_t)v);
    if (segk[b] > 1 && key > far[b]) atomicMax(&far[b], key);
}

__global__ void k_gp_far_src(int32_t nparts, const int32_t *segk, const unsigned long long *far, int32_t *src) {
    const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nparts && segk[b] > 1) src[b] = (int32_t)(~(uint32_t)(far[b] & 0xffffffffull));
}

__global__ void k_gp_keys(int64_t n, const int32_t *label, const uint32_t *dist, unsigned long long *key,
                          int32_t *idx) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    key[v] = ((unsigned long long)(uint32_t)label[v] << 32) | dist[v];
    idx[v] = (int32_t)v;
}

// the segment of label b starts at sorted position b*S: every smaller label
// heads a segment whose vertices all come first
__global__ void k_gp_split(int64_t n, int32_t S, const int32_t *sorted, const int32_t *segk, int32_t *label) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t v = sorted[i];
    const int32_t b = label[v];
    const int32_t k = segk[b];
    if (k <= 1) return;
    const int32_t k0 = k / 2;
    label[v] = (i - (int64_t)b * S) < (int64_t)k0 * S ? b : b + k0;
}

__global__ void k_gp_label_keys(int64_t n, const int32_t *label, uint32_t *key, int32_t *idx) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    key[v] = (uint32_t)label[v];
    idx[v] = (int32_t)v;
}

__global__ void k_gp_perm(int64_t n, const int32_t *sorted, int32_t *new2old, int32_t *old2new) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t v = sorted[i];
    new2old[i] = v;
    old2new[v] = (int32_t)i;
}

int bits_for(uint64_t x) {
    int b = 0;
    while (b < 64 && (x >> b) != 0) ++b;
    return b < 1 ? 1 : b;
}

}  // namespace

int graph_partition(dd_ctx *h, const int32_t *ptr, const int32_t *col, hipStream_t st) {
    const int64_t n = h->n;
    const int32_t S = h->S, nparts = h->nsub;
    std::vector<void *> tmp;
    auto get = [&](auto **p, int64_t count) -> hipError_t {
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, (size_t)std::max<int64_t>(count, 1) * sizeof(**p));
        if (e == hipSuccess) {
            tmp.push_back(q);
            *p = static_cast<std::remove_reference_t<decltype(*p)>>(q);
        }
        return e;
    };
    auto done = [&](int rc) {
        for (void *q : tmp) (void)hipFree(q);
        return rc;
    };
#define GCHK(x)                                                                   \
    do {                                                                          \
        hipError_t e_ = (x);                                                      \
        if (e_ != hipSuccess) {                                                   \
            (void)hipGetLastError();                                              \
            h->fail(DD_EHIP, "graph partition: %s: %s", #x, hipGetErrorString(e_)); \
            return done(DD_EHIP);                                                 \
        }                                                                         \
    } while (0)
    int32_t *label = h->part_id, *segk = nullptr, *src = nullptr, *idx = nullptr, *sorted = nullptr,
            *changed = nullptr;
    uint32_t *dist = nullptr;
    unsigned long long *key = nullptr, *key2 = nullptr, *far = nullptr;
    GCHK(get(&segk, nparts));
    GCHK(get(&src, nparts));
    GCHK(get(&far, nparts));
    GCHK(get(&dist, n));
    GCHK(get(&key, n));
    GCHK(get(&key2, n));
    GCHK(get(&idx, n));
    GCHK(get(&sorted, n));
    GCHK(get(&changed, kLevelBatch));
    size_t temp_bytes = 0, temp32 = 0;
    GCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, key, key2, idx, sorted, (int)n, 0, 64, st));
    GCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, temp32, reinterpret_cast<uint32_t *>(key),
                                           reinterpret_cast<uint32_t *>(key2), idx, sorted, (int)n, 0, 32, st));
    temp_bytes = std::max(temp_bytes, temp32);
    void *temp = nullptr;
    GCHK(get(reinterpret_cast<unsigned char **>(&temp), (int64_t)temp_bytes));
    const int end_bit = 32 + bits_for((uint64_t)nparts);

    std::vector<int32_t> kh(nparts, 0), next(nparts, 0);
    kh[0] = nparts;
    k_gp_fill<<<blocks(n), kT, 0, st>>>(n, label, 0);
    GCHK(hipGetLastError());

    auto bfs = [&]() -> hipError_t {
        k_gp_src<<<blocks(n), kT, 0, st>>>(n, label, segk, src, dist);
        hipError_t e = hipGetLastError();
        for (uint32_t d = 0; e == hipSuccess && d < (uint32_t)n; d += kLevelBatch) {
            k_gp_fill<<<1, kT, 0, st>>>(kLevelBatch, changed, 0);
            for (int j = 0; j < kLevelBatch; ++j)
                k_gp_level<<<blocks(n), kT, 0, st>>>(n, ptr, col, label, d + j, dist, changed + j);
            int32_t last = 0;
            if ((e = hipGetLastError()) != hipSuccess) break;
            if ((e = hipMemcpyAsync(&last, changed + kLevelBatch - 1, sizeof(int32_t), hipMemcpyDeviceToHost,
                                    st)) != hipSuccess)
                break;
            if ((e = hipStreamSynchronize(st)) != hipSuccess) break;
            if (!last) break;  // no vertex at distance d + kLevelBatch: every segment is exhausted
        }
        return e;
    };

    for (;;) {
        bool split = false;
        for (int32_t b = 0; b < nparts; ++b) split = split || kh[b] > 1;
        if (!split) break;
        GCHK(hipMemcpyAsync(segk, kh.data(), sizeof(int32_t) * nparts, hipMemcpyHostToDevice, st));
        k_gp_fill<<<blocks(nparts), kT, 0, st>>>(nparts, src, 0x7fffffff);
        k_gp_vmin<<<blocks(n), kT, 0, st>>>(n, label, segk, src);
        GCHK(hipGetLastError());
        GCHK(bfs());
        k_gp_fill64<<<blocks(nparts), kT, 0, st>>>(nparts, far);
        k_gp_far<<<blocks(n), kT, 0, st>>>(n, label, segk, dist, far);
        k_gp_far_src<<<blocks(nparts), kT, 0, st>>>(nparts, segk, far, src);
        GCHK(hipGetLastError());
        GCHK(bfs());
        k_gp_keys<<<blocks(n), kT, 0, st>>>(n, label, dist, key, idx);
        GCHK(hipGetLastError());
        GCHK(hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, key, key2, idx, sorted, (int)n, 0, end_bit, st));
        k_gp_split<<<blocks(n), kT, 0, st>>>(n, S, sorted, segk, label);
        GCHK(hipGetLastError());
        std::fill(next.begin(), next.end(), 0);
        for (int32_t b = 0; b < nparts; ++b) {
            if (kh[b] == 1) next[b] = 1;
            if (kh[b] > 1) {
                next[b] = kh[b] / 2;
                next[b + kh[b] / 2] = kh[b] - kh[b] / 2;
            }
        }
        kh.swap(next);
    }
    // renumber: stable sort of the vertices by label
    uint32_t *lkey = reinterpret_cast<uint32_t *>(key), *lkey2 = reinterpret_cast<uint32_t *>(key2);
    k_gp_label_keys<<<blocks(n), kT, 0, st>>>(n, label, lkey, idx);
    GCHK(hipGetLastError());
    GCHK(hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, lkey, lkey2, idx, sorted, (int)n, 0,
                                           bits_for((uint64_t)nparts), st));
    k_gp_perm<<<blocks(n), kT, 0, st>>>(n, sorted, h->new2old, h->old2new);
    GCHK(hipGetLastError());
    GCHK(hipStreamSynchronize(st));
#undef GCHK
    return done(DD_OK);
}

}  // namespace ddilu
