// Cell list for the real-space pair loop: positions are reduced into [0, L)^3,
// binned into nc^3 cubic cells of side h = L / nc >= r_c / 2, and copied into
// cell-sorted 32-byte records (x, y, z, q).  Inside a cell particles keep their
// input order, so every later floating-point sum runs in a fixed order and
// results are bitwise reproducible.
//
// The paper's local PairLoop builds an equivalent cell structure on the CPU
// (section 2.2); here it is four short kernels:
//   bin      : wrap, cell id, per-cell counts (integer atomics), charge sums,
//              non-finite detection;
//   scan     : exclusive scan of the counts (tile totals, then one block per
//              tile), pair-loop work items, total charge;
//   scatter  : slot claim inside each cell (order not yet deterministic);
//   cellsort : per cell, restore input order (rank, or sort the indices) and
//              write the sorted records.
// A small system (at most 512 particles and 4096 cells) takes all four steps
// in one workgroup (k_cells_small), with the same results.
#include <algorithm>

#include "ewald_internal.h"

namespace ewk {

namespace {

constexpr int kBinThreads = 256;

__device__ inline int cell_coord(double w, double L, int nc)
{
    int c = (int)(w * (double)nc / L);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__device__ __forceinline__ void bin_body(int bx, int by, int64_t n, double L, int nc, const double *__restrict__ pos,
                                         const double *__restrict__ q, int *__restrict__ cell_of,
                                         int *__restrict__ counts, double *__restrict__ qpart, int *__restrict__ status)
{
    __shared__ double s_q[kBinThreads];
    __shared__ double s_q2[kBinThreads];
    const int64_t i = (int64_t)bx * kBinThreads + threadIdx.x;
    double qi = 0.0;
    if (i < n) {
        const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
        qi = q[i];
        const bool fin = isfinite(x) && isfinite(y) && isfinite(z) && isfinite(qi);
        int c = 0;
        if (fin) {
            c = (cell_coord(wrap_coord(x, L), L, nc) * nc + cell_coord(wrap_coord(y, L), L, nc)) * nc +
                cell_coord(wrap_coord(z, L), L, nc);
        } else {
            atomicOr(status, 1);
        }
        cell_of[i] = c;
        atomicAdd(&counts[c], 1);
    }
    s_q[threadIdx.x] = qi;
    s_q2[threadIdx.x] = qi * qi;
    __syncthreads();
    for (int w = kBinThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s_q[threadIdx.x] += s_q[threadIdx.x + w];
            s_q2[threadIdx.x] += s_q2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        qpart[2 * bx] = s_q[0];
        qpart[2 * bx + 1] = s_q2[0];
    }
}

struct KBin {
    static constexpr int kThreads = kBinThreads;
    static constexpr int kWavesPerEu = 1;
    int64_t n;
    double L;
    int nc;
    const double *pos;
    const double *q;
    int *cell_of;
    int *counts;
    double *qpart;
    int *status;
    __device__ void run(int bx, int by) const { bin_body(bx, by, n, L, nc, pos, q, cell_of, counts, qpart, status); }
    hipError_t one(hipStream_t s, dim3 grid, int threads, size_t smem) const;
};

__global__ __launch_bounds__(kBinThreads) void k_bin(int64_t n, double L, int nc, const double *__restrict__ pos,
                                                     const double *__restrict__ q, int *__restrict__ cell_of,
                                                     int *__restrict__ counts, double *__restrict__ qpart,
                                                     int *__restrict__ status)
{
    bin_body(blockIdx.x, blockIdx.y, n, L, nc, pos, q, cell_of, counts, qpart, status);
}

hipError_t KBin::one(hipStream_t s, dim3 grid, int threads, size_t smem) const
{
    hipLaunchKernelGGL((k_bin), grid, dim3(threads), smem, s, n, L, nc, pos, q, cell_of, counts, qpart, status);
    return hipGetLastError();
}

constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;                           // cells per thread
constexpr int kScanTile = kScanThreads * kScanPer;    // cells per block

// Counts of the kScanPer consecutive cells c0 .. c0 + kScanPer - 1 (zero past
// ncell): one 16-byte load when the whole group lies inside the array.
__device__ inline int4 load_counts(const int *__restrict__ counts, int c0, int ncell)
{
    if (c0 + kScanPer <= ncell) return *reinterpret_cast<const int4 *>(counts + c0);
    int4 v = {0, 0, 0, 0};
    if (c0 < ncell) v.x = counts[c0];
    if (c0 + 1 < ncell) v.y = counts[c0 + 1];
    if (c0 + 2 < ncell) v.z = counts[c0 + 2];
    return v;
}

__device__ inline int items_of(int k) { return (k + kPairHome - 1) / kPairHome; }

// Block-wide sums (sum over all threads) of two integers.
__device__ inline int2 block_sum2(int a, int b, int2 *s_w)
{
    const int lane = (int)threadIdx.x % kLanes, wave = (int)threadIdx.x / kLanes;
#pragma unroll
    for (int d = kLanes / 2; d > 0; d >>= 1) {
        a += __shfl_xor(a, d);
        b += __shfl_xor(b, d);
    }
    if (lane == 0) s_w[wave] = make_int2(a, b);
    __syncthreads();
    int2 t = {0, 0};
#pragma unroll
    for (int w = 0; w < kScanThreads / kLanes; ++w) {
        t.x += s_w[w].x;
        t.y += s_w[w].y;
    }
    __syncthreads();  // s_w may be reused
    return t;
}

// Pass 1 of the cell scan, one block per tile of kScanTile cells: the tile's
// particle and pair-work-item totals.  Block n_tiles (the last one) instead
// reduces the per-block charge sums of the binning into scalars[0] = Q and
// scalars[1] = sum q^2, in a fixed order (contiguous ranges, then a fixed tree).
__device__ __forceinline__ void scan_tiles_body(int bx, int by, int ncell, int n_tiles, const int *__restrict__ counts,
                                                int2 *__restrict__ tile_sums, const double *__restrict__ qpart,
                                                int n_qblocks, double *__restrict__ scalars)
{
    __shared__ int2 s_w[kScanThreads / kLanes];
    __shared__ double s_a[kScanThreads];
    __shared__ double s_b[kScanThreads];
    const int t = (int)threadIdx.x;
    if ((int)bx < n_tiles) {
        const int4 v = load_counts(counts, (int)bx * kScanTile + t * kScanPer, ncell);
        const int2 tot = block_sum2(v.x + v.y + v.z + v.w, items_of(v.x) + items_of(v.y) + items_of(v.z) + items_of(v.w),
                                    s_w);
        if (t == 0) tile_sums[bx] = tot;
        return;
    }
    const int qper = (n_qblocks + kScanThreads - 1) / kScanThreads;
    double a = 0.0, b = 0.0;
    for (int k = t * qper; k < (t + 1) * qper && k < n_qblocks; ++k) {
        a += qpart[2 * k];
        b += qpart[2 * k + 1];
    }
    s_a[t] = a;
    s_b[t] = b;
    __syncthreads();
    for (int w = kScanThreads / 2; w > 0; w >>= 1) {
        if (t < w) {
            s_a[t] += s_a[t + w];
            s_b[t] += s_b[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        scalars[0] = s_a[0];
        scalars[1] = s_b[0];
    }
}

struct KScanTiles {
    static constexpr int kThreads = kScanThreads;
    static constexpr int kWavesPerEu = 1;
    int ncell;
    int n_tiles;
    const int *counts;
    int2 *tile_sums;
    const double *qpart;
    int n_qblocks;
    double *scalars;
    __device__ void run(int bx, int by) const
    {
        scan_tiles_body(bx, by, ncell, n_tiles, counts, tile_sums, qpart, n_qblocks, scalars);
    }
    hipError_t one(hipStream_t s, dim3 grid, int threads, size_t smem) const;
};

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(int ncell, int n_tiles, const int *__restrict__ counts,
                                                             int2 *__restrict__ tile_sums,
                                                             const double *__restrict__ qpart, int n_qblocks,
                                                             double *__restrict__ scalars)
{
    scan_tiles_body(blockIdx.x, blockIdx.y, ncell, n_tiles, counts, tile_sums, qpart, n_qblocks, scalars);
}

hipError_t KScanTiles::one(hipStream_t s, dim3 grid, int threads, size_t smem) const
{
    hipLaunchKernelGGL((k_scan_tiles), grid, dim3(threads), smem, s, ncell, n_tiles, counts, tile_sums, qpart,
                       n_qblocks, scalars);
    return hipGetLastError();
}

// Pass 2, one block per tile: the tile's offset is the sum of the earlier
// tiles' totals; an exclusive scan of the counts inside the tile (wave
// shuffles, then the waves' totals) gives cell_start, and the pair-loop work
// items (one per cell and kPairHome home particles, in cell order) are written
// at the matching item offsets as (cell, offset of the first home particle).  Counts and fill are cleared for the next
// evaluation.  The last block writes cell_start[ncell] and the item count.
__device__ __forceinline__ void scan_cells_body(int bx, int by, int ncell, int n_tiles, int *__restrict__ counts,
                                                int *__restrict__ fill, const int2 *__restrict__ tile_sums,
                                                int *__restrict__ cell_start, int *__restrict__ item_cell,
                                                int *__restrict__ item_off, int *__restrict__ n_items)
{
    __shared__ int2 s_w[kScanThreads / kLanes];
    const int t = (int)threadIdx.x, lane = t % kLanes, wave = t / kLanes;
    const int b = (int)bx;
    int pa = 0, pb = 0;
    for (int k = t; k < b; k += kScanThreads) {
        const int2 v = tile_sums[k];
        pa += v.x;
        pb += v.y;
    }
    const int2 base = block_sum2(pa, pb, s_w);
    const int c0 = b * kScanTile + t * kScanPer;
    const int4 v = load_counts(counts, c0, ncell);
    const int cnt[kScanPer] = {v.x, v.y, v.z, v.w};
    int la = 0, lb = 0;
#pragma unroll
    for (int u = 0; u < kScanPer; ++u) {
        la += cnt[u];
        lb += items_of(cnt[u]);
    }
    // inclusive scans inside each wave
    int ia = la, ib = lb;
#pragma unroll
    for (int d = 1; d < kLanes; d <<= 1) {
        const int xa = __shfl_up(ia, d), xb = __shfl_up(ib, d);
        if (lane >= d) {
            ia += xa;
            ib += xb;
        }
    }
    if (lane == kLanes - 1) s_w[wave] = make_int2(ia, ib);
    __syncthreads();
    int wa = 0, wb = 0, ta = 0, tb = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / kLanes; ++w) {
        const int2 x = s_w[w];
        if (w < wave) {
            wa += x.x;
            wb += x.y;
        }
        ta += x.x;
        tb += x.y;
    }
    int run = base.x + wa + ia - la;
    int irun = base.y + wb + ib - lb;
#pragma unroll
    for (int u = 0; u < kScanPer; ++u) {
        const int c = c0 + u;
        if (c < ncell) {
            cell_start[c] = run;
            run += cnt[u];
            for (int o = 0; o < cnt[u]; o += kPairHome) {
                item_cell[irun] = c;
                item_off[irun] = o;
                ++irun;
            }
            counts[c] = 0;
            fill[c] = 0;
        }
    }
    if (b == n_tiles - 1 && t == 0) {
        cell_start[ncell] = base.x + ta;
        *n_items = base.y + tb;
    }
}

struct KScanCells {
    static constexpr int kThreads = kScanThreads;
    static constexpr int kWavesPerEu = 1;
    int ncell;
    int n_tiles;
    int *counts;
    int *fill;
    const int2 *tile_sums;
    int *cell_start;
    int *item_cell;
    int *item_off;
    int *n_items;
    __device__ void run(int bx, int by) const
    {
        scan_cells_body(bx, by, ncell, n_tiles, counts, fill, tile_sums, cell_start, item_cell, item_off, n_items);
    }
    hipError_t one(hipStream_t s, dim3 grid, int threads, size_t smem) const;
};

__global__ __launch_bounds__(kScanThreads) void k_scan_cells(int ncell, int n_tiles, int *__restrict__ counts,
                                                             int *__restrict__ fill, const int2 *__restrict__ tile_sums,
                                                             int *__restrict__ cell_start, int *__restrict__ item_cell,
                                                             int *__restrict__ item_off, int *__restrict__ n_items)
{
    scan_cells_body(blockIdx.x, blockIdx.y, ncell, n_tiles, counts, fill, tile_sums, cell_start, item_cell, item_off,
                    n_items);
}

hipError_t KScanCells::one(hipStream_t s, dim3 grid, int threads, size_t smem) const
{
    hipLaunchKernelGGL((k_scan_cells), grid, dim3(threads), smem, s, ncell, n_tiles, counts, fill, tile_sums,
                       cell_start, item_cell, item_off, n_items);
    return hipGetLastError();
}

__device__ __forceinline__ void scatter_body(int bx, int by, int64_t n, const int *__restrict__ cell_of,
                                             const int *__restrict__ cell_start, int *__restrict__ fill,
                                             int *__restrict__ tmp_idx)
{
    const int64_t i = (int64_t)bx * 256 + threadIdx.x;
    if (i >= n) return;
    const int c = cell_of[i];
    const int slot = cell_start[c] + atomicAdd(&fill[c], 1);
    tmp_idx[slot] = (int)i;
}

struct KScatter {
    static constexpr int kThreads = 256;
    static constexpr int kWavesPerEu = 1;
    int64_t n;
    const int *cell_of;
    const int *cell_start;
    int *fill;
    int *tmp_idx;
    __device__ void run(int bx, int by) const { scatter_body(bx, by, n, cell_of, cell_start, fill, tmp_idx); }
    hipError_t one(hipStream_t s, dim3 grid, int threads, size_t smem) const;
};

__global__ __launch_bounds__(256) void k_scatter(int64_t n, const int *__restrict__ cell_of,
                                                 const int *__restrict__ cell_start, int *__restrict__ fill,
                                                 int *__restrict__ tmp_idx)
{
    scatter_body(blockIdx.x, blockIdx.y, n, cell_of, cell_start, fill, tmp_idx);
}

hipError_t KScatter::one(hipStream_t s, dim3 grid, int threads, size_t smem) const
{
    hipLaunchKernelGGL((k_scatter), grid, dim3(threads), smem, s, n, cell_of, cell_start, fill, tmp_idx);
    return hipGetLastError();
}

constexpr int kSortThreads = 128;
constexpr int kSortLds = 2048;
constexpr int kSortRank = 256;  // cells up to this size are ranked directly

// Ascending bitonic sort of v[0, cnt) by one workgroup, in the variant whose
// every compare-exchange puts the smaller value at the lower index (the first
// step of each merge compares mirrored positions of a block, the later steps
// positions j apart).  Positions past cnt stand for +infinity, so a pair whose
// upper position is past cnt never exchanges and is skipped: no padding is
// stored.  O(cnt log^2 cnt) work, (log2 P)(log2 P + 1) / 2 barriers for P the
// power of two at or above cnt.  V is a pointer to LDS or to global memory
// (the workgroup barrier orders both).
template <int THREADS, typename V>
__device__ inline void bitonic_sort_block(V v, int cnt)
{
    int P = 1;
    while (P < cnt) P <<= 1;
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = (int)threadIdx.x; t < P / 2; t += THREADS) {
                const int blk = t / j, o = t % j;
                int lo, hi;
                if (j == k >> 1) {  // mirrored positions of a block of k
                    lo = blk * k + o;
                    hi = blk * k + k - 1 - o;
                } else {
                    lo = blk * 2 * j + o;
                    hi = lo + j;
                }
                if (hi < cnt) {
                    const int x = v[lo], y = v[hi];
                    if (y < x) {
                        v[lo] = y;
                        v[hi] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// One workgroup per cell.  The scatter above claimed slots in arbitrary order;
// the cell's entries go back to input order: an entry's rank is the number of
// entries of the cell with a smaller input index (cells of at most kSortRank
// entries), or the cell's indices are sorted (bitonic, in LDS up to kSortLds
// entries, in place in tmp_idx beyond), so that the rank is the position.
// Either way the order is the same, and O(cnt log^2 cnt) bounds the work of
// a crowded cell.
__device__ __forceinline__ void cellsort_body(int bx, int by, double L, const int *__restrict__ cell_start,
                                              int *__restrict__ tmp_idx, const double *__restrict__ pos,
                                              const double *__restrict__ q, int *__restrict__ perm, d4 *__restrict__ pq)
{
    __shared__ int s_idx[kSortLds];
    const int c = bx;
    const int start = cell_start[c];
    const int cnt = cell_start[c + 1] - start;
    const bool in_lds = cnt <= kSortLds;  // uniform over the workgroup
    const bool ranked = cnt <= kSortRank;
    if (in_lds) {
        for (int e = threadIdx.x; e < cnt; e += kSortThreads) s_idx[e] = tmp_idx[start + e];
    }
    __syncthreads();
    if (!ranked) {
        if (in_lds)
            bitonic_sort_block<kSortThreads>(s_idx, cnt);
        else
            bitonic_sort_block<kSortThreads>(tmp_idx + start, cnt);
    }
    for (int e = threadIdx.x; e < cnt; e += kSortThreads) {
        const int mine = in_lds ? s_idx[e] : tmp_idx[start + e];
        int rank = e;
        if (ranked) {
            rank = 0;
            for (int f = 0; f < cnt; ++f) rank += s_idx[f] < mine;
        }
        const int s = start + rank;
        perm[s] = mine;
        d4 r;
        r.a = wrap_coord(pos[3 * (int64_t)mine], L);
        r.b = wrap_coord(pos[3 * (int64_t)mine + 1], L);
        r.c = wrap_coord(pos[3 * (int64_t)mine + 2], L);
        r.d = q[mine];
        pq[s] = r;
    }
}

struct KCellSort {
    static constexpr int kThreads = kSortThreads;
    static constexpr int kWavesPerEu = 1;
    double L;
    const int *cell_start;
    int *tmp_idx;
    const double *pos;
    const double *q;
    int *perm;
    d4 *pq;
    __device__ void run(int bx, int by) const { cellsort_body(bx, by, L, cell_start, tmp_idx, pos, q, perm, pq); }
    hipError_t one(hipStream_t s, dim3 grid, int threads, size_t smem) const;
};

__global__ __launch_bounds__(kSortThreads) void k_cellsort(double L, const int *__restrict__ cell_start,
                                                           int *__restrict__ tmp_idx, const double *__restrict__ pos,
                                                           const double *__restrict__ q, int *__restrict__ perm,
                                                           d4 *__restrict__ pq)
{
    cellsort_body(blockIdx.x, blockIdx.y, L, cell_start, tmp_idx, pos, q, perm, pq);
}

hipError_t KCellSort::one(hipStream_t s, dim3 grid, int threads, size_t smem) const
{
    hipLaunchKernelGGL((k_cellsort), grid, dim3(threads), smem, s, L, cell_start, tmp_idx, pos, q, perm, pq);
    return hipGetLastError();
}

constexpr int kSmallThreads = 1024;
constexpr int kSmallIndexBits = 11;  // index bits of a key (>= log2 kSmallCellsMaxN)

// Tree over the kBinThreads values of each group of kBinThreads threads, in the
// order of k_bin's tree (t += t + w for w = 128, 64, ..., 1): the two widest
// steps through LDS, the rest with shuffles inside the wave (lane t receives
// lane t + w), so fewer barriers give the same sums.
__device__ inline void group_tree256(double &a, double &b, double *s_a, double *s_b)
{
    const int t = (int)threadIdx.x, g = t % kBinThreads;
    s_a[t] = a;
    s_b[t] = b;
    __syncthreads();
    if (g < 128) {
        s_a[t] += s_a[t + 128];
        s_b[t] += s_b[t + 128];
    }
    __syncthreads();
    if (g < 64) {
        s_a[t] += s_a[t + 64];
        s_b[t] += s_b[t + 64];
    }
    __syncthreads();
    a = s_a[t];
    b = s_b[t];
#pragma unroll
    for (int w = 32; w > 0; w >>= 1) {
        const double xa = __shfl_down(a, w), xb = __shfl_down(b, w);
        if (g < w) {
            a += xa;
            b += xb;
        }
    }
    __syncthreads();  // s_a, s_b may be refilled
}

// The whole cell list of a small system (n <= kSmallCellsMaxN, ncell <=
// kSmallCellsMaxCells) in one workgroup, with the outputs of the four kernels
// above bit for bit: the same cells, charge sums in the same order (trees over
// 256-particle chunks as k_bin, then the tree of k_scan_tiles), the same
// cell_start and pair-work items, and particles in cell order, input order
// inside a cell.  A particle's place is the rank of its key cell << 11 | index
// among all keys (counted against the keys in LDS, no sort and no barriers).
// One launch instead of four, which is most of a small system's real-space
// path.
__device__ __forceinline__ void cells_small_body(int bx, int by, int n, double L, int nc,
                                                 const double *__restrict__ pos, const double *__restrict__ q,
                                                 int *__restrict__ cell_start, int *__restrict__ item_cell,
                                                 int *__restrict__ item_off, int *__restrict__ n_items,
                                                 double *__restrict__ scalars, int *__restrict__ perm,
                                                 d4 *__restrict__ pq, int *__restrict__ status)
{
    __shared__ int s_key[kSmallCellsMaxN];
    __shared__ d4 s_rec[kSmallCellsMaxN];  // wrapped position and charge
    __shared__ int s_cnt[kSmallCellsMaxCells];
    __shared__ double s_a[kSmallThreads], s_b[kSmallThreads];
    __shared__ double s_qp[2 * (kSmallCellsMaxN / kBinThreads)];
    __shared__ int2 s_w[kSmallThreads / kLanes];
    const int t = (int)threadIdx.x, lane = t % kLanes, wave = t / kLanes;
    const int ncell = nc * nc * nc;
    const int nq = (n + kBinThreads - 1) / kBinThreads;
    for (int c = t; c < ncell; c += kSmallThreads) s_cnt[c] = 0;
    __syncthreads();
    // cells, keys, counts and records; charge partials of each chunk of kBinThreads
    for (int base = 0; base < n; base += kSmallThreads) {
        const int i = base + t;
        double qi = 0.0;
        if (i < n) {
            const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
            qi = q[i];
            const bool fin = isfinite(x) && isfinite(y) && isfinite(z) && isfinite(qi);
            d4 r;
            r.a = wrap_coord(x, L);
            r.b = wrap_coord(y, L);
            r.c = wrap_coord(z, L);
            r.d = qi;
            int c = 0;
            if (fin)
                c = (cell_coord(r.a, L, nc) * nc + cell_coord(r.b, L, nc)) * nc + cell_coord(r.c, L, nc);
            else
                atomicOr(status, 1);
            s_key[i] = (c << kSmallIndexBits) | i;
            s_rec[i] = r;
            atomicAdd(&s_cnt[c], 1);
        }
        double a = qi, b = qi * qi;
        group_tree256(a, b, s_a, s_b);
        const int blk = (base + t) / kBinThreads;
        if (t % kBinThreads == 0 && blk < nq) {
            s_qp[2 * blk] = a;
            s_qp[2 * blk + 1] = b;
        }
    }
    __syncthreads();
    // Q and sum q^2 (k_scan_tiles' last block: chunk k on thread k, then a tree)
    {
        double a = 0.0, b = 0.0;
        if (t < nq) {
            a += s_qp[2 * t];
            b += s_qp[2 * t + 1];
        }
        group_tree256(a, b, s_a, s_b);
        if (t == 0) {
            scalars[0] = a;
            scalars[1] = b;
        }
    }
    // exclusive scans of the counts and of the pair-work items, kScanPer cells
    // per thread (ncell <= kScanPer kSmallThreads)
    const int c0 = t * kScanPer;
    int cnt[kScanPer];
    int la = 0, lb = 0;
#pragma unroll
    for (int u = 0; u < kScanPer; ++u) {
        cnt[u] = c0 + u < ncell ? s_cnt[c0 + u] : 0;
        la += cnt[u];
        lb += items_of(cnt[u]);
    }
    int ia = la, ib = lb;
#pragma unroll
    for (int d = 1; d < kLanes; d <<= 1) {
        const int xa = __shfl_up(ia, d), xb = __shfl_up(ib, d);
        if (lane >= d) {
            ia += xa;
            ib += xb;
        }
    }
    if (lane == kLanes - 1) s_w[wave] = make_int2(ia, ib);
    __syncthreads();
    int wa = 0, wb = 0, ta = 0, tb = 0;
#pragma unroll
    for (int w = 0; w < kSmallThreads / kLanes; ++w) {
        const int2 x = s_w[w];
        if (w < wave) {
            wa += x.x;
            wb += x.y;
        }
        ta += x.x;
        tb += x.y;
    }
    int run = wa + ia - la;
    int irun = wb + ib - lb;
#pragma unroll
    for (int u = 0; u < kScanPer; ++u) {
        const int c = c0 + u;
        if (c < ncell) {
            cell_start[c] = run;
            run += cnt[u];
            for (int o = 0; o < cnt[u]; o += kPairHome) {
                item_cell[irun] = c;
                item_off[irun] = o;
                ++irun;
            }
        }
    }
    if (t == 0) {
        cell_start[ncell] = ta;
        *n_items = tb;
    }
    // records in cell order: the rank of each key among all keys
    for (int i = t; i < n; i += kSmallThreads) {
        const int mine = s_key[i];
        int rank = 0;
        for (int j = 0; j < n; ++j) rank += s_key[j] < mine;
        perm[rank] = i;
        pq[rank] = s_rec[i];
    }
}

struct KCellsSmall {
    static constexpr int kThreads = kSmallThreads;
    static constexpr int kWavesPerEu = 1;
    int n;
    double L;
    int nc;
    const double *pos;
    const double *q;
    int *cell_start;
    int *item_cell;
    int *item_off;
    int *n_items;
    double *scalars;
    int *perm;
    d4 *pq;
    int *status;
    __device__ void run(int bx, int by) const
    {
        cells_small_body(bx, by, n, L, nc, pos, q, cell_start, item_cell, item_off, n_items, scalars, perm, pq, status);
    }
    hipError_t one(hipStream_t s, dim3 grid, int threads, size_t smem) const;
};

__global__ __launch_bounds__(kSmallThreads) void k_cells_small(int n, double L, int nc, const double *__restrict__ pos,
                                                               const double *__restrict__ q,
                                                               int *__restrict__ cell_start,
                                                               int *__restrict__ item_cell, int *__restrict__ item_off,
                                                               int *__restrict__ n_items, double *__restrict__ scalars,
                                                               int *__restrict__ perm, d4 *__restrict__ pq,
                                                               int *__restrict__ status)
{
    cells_small_body(blockIdx.x, blockIdx.y, n, L, nc, pos, q, cell_start, item_cell, item_off, n_items, scalars, perm,
                     pq, status);
}

hipError_t KCellsSmall::one(hipStream_t s, dim3 grid, int threads, size_t smem) const
{
    hipLaunchKernelGGL((k_cells_small), grid, dim3(threads), smem, s, n, L, nc, pos, q, cell_start, item_cell, item_off,
                       n_items, scalars, perm, pq, status);
    return hipGetLastError();
}

// Clears `words` 16-byte words (the counters and padding an evaluation expects
// at zero, when its buffers come from memory another evaluation used).
__device__ __forceinline__ void zero_body(int bx, uint4 *__restrict__ p, int64_t words, int blocks)
{
    const uint4 z = {0u, 0u, 0u, 0u};
    for (int64_t i = (int64_t)bx * 256 + threadIdx.x; i < words; i += (int64_t)blocks * 256) p[i] = z;
}

struct KZero {
    static constexpr int kThreads = 256;
    static constexpr int kWavesPerEu = 1;
    uint4 *p;
    int64_t words;
    int blocks;  // the launch's grid
    __device__ void run(int bx, int) const { zero_body(bx, p, words, blocks); }
    hipError_t one(hipStream_t s, dim3 grid, int threads, size_t smem) const;
};

__global__ __launch_bounds__(256) void k_zero(uint4 *__restrict__ p, int64_t words, int blocks)
{
    zero_body(blockIdx.x, p, words, blocks);
}

hipError_t KZero::one(hipStream_t s, dim3 grid, int threads, size_t smem) const
{
    hipLaunchKernelGGL(k_zero, grid, dim3(threads), smem, s, p, words, blocks);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_zero(hipStream_t s, void *p, size_t bytes)
{
    const int64_t words = (int64_t)(bytes / sizeof(uint4));
    if (words == 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>(ceil_div(words, 256), 2048);
    return launch(s, dim3(blocks), 256, 0, KZero{static_cast<uint4 *>(p), words, blocks});
}

hipError_t launch_bin(hipStream_t s, const CellArgs &a, const double *pos, const double *q, int *cell_of,
                      int *counts, double *qpart, int *status)
{
    return launch(s, dim3(ceil_div(a.n, kBinThreads)), kBinThreads, 0,
                  KBin{a.n, a.L, a.nc, pos, q, cell_of, counts, qpart, status});
}

hipError_t launch_scan(hipStream_t s, const CellArgs &a, int *counts, int *fill, int *cell_start,
                       const double *qpart, int n_qblocks, double *scalars, int2 *tile_sums, int *item_cell,
                       int *item_off, int *n_items)
{
    const int n_tiles = scan_tiles(a.ncell);
    const hipError_t e = launch(s, dim3(n_tiles + 1), kScanThreads, 0,
                                KScanTiles{a.ncell, n_tiles, counts, tile_sums, qpart, n_qblocks, scalars});
    if (e != hipSuccess) return e;
    return launch(s, dim3(n_tiles), kScanThreads, 0,
                  KScanCells{a.ncell, n_tiles, counts, fill, tile_sums, cell_start, item_cell, item_off, n_items});
}

int scan_tiles(int ncell) { return ceil_div(ncell, kScanTile); }

hipError_t launch_scatter(hipStream_t s, const CellArgs &a, const int *cell_of, const int *cell_start,
                          int *fill, int *tmp_idx)
{
    return launch(s, dim3(ceil_div(a.n, 256)), 256, 0, KScatter{a.n, cell_of, cell_start, fill, tmp_idx});
}

hipError_t launch_cellsort(hipStream_t s, const CellArgs &a, const int *cell_start, int *tmp_idx,
                           const double *pos, const double *q, int *perm, d4 *pq)
{
    return launch(s, dim3(a.ncell), kSortThreads, 0, KCellSort{a.L, cell_start, tmp_idx, pos, q, perm, pq});
}

int bin_blocks(int64_t n) { return ceil_div(n, kBinThreads); }

bool cells_small(const CellArgs &a) { return a.n <= kSmallCellsMaxN && a.ncell <= kSmallCellsMaxCells; }

hipError_t launch_cells_small(hipStream_t s, const CellArgs &a, const double *pos, const double *q, int *cell_start,
                              int *item_cell, int *item_off, int *n_items, double *scalars, int *perm, d4 *pq,
                              int *status)
{
    return launch(s, dim3(1), kSmallThreads, 0,
                  KCellsSmall{(int)a.n, a.L, a.nc, pos, q, cell_start, item_cell, item_off, n_items, scalars, perm,
                              pq, status});
}

}  // namespace ewk
