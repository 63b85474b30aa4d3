// Cell list for the real-space pair loop: positions are reduced into [0, L)^3,
// binned into nc^3 cubic cells of side h = L / nc >= r_c, and copied into
// cell-sorted 32-byte records (x, y, z, q).  Inside a cell particles keep their
// input order, so every later floating-point sum runs in a fixed order and
// results are bitwise reproducible.
//
// The paper's local PairLoop builds an equivalent cell structure on the CPU
// (section 2.2); here it is four short kernels:
//   bin      : wrap, cell id, per-cell counts (integer atomics), charge sums,
//              non-finite detection;
//   scan     : exclusive scan of the counts (one workgroup), total charge;
//   scatter  : slot claim inside each cell (order not yet deterministic);
//   cellsort : per cell, rank by input index and write the sorted records.
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

__global__ __launch_bounds__(kBinThreads) void k_bin(int64_t n, double L, int nc,
                                                     const double *__restrict__ pos,
                                                     const double *__restrict__ q,
                                                     int *__restrict__ cell_of, int *__restrict__ counts,
                                                     double *__restrict__ qpart, int *__restrict__ status)
{
    __shared__ double s_q[kBinThreads];
    __shared__ double s_q2[kBinThreads];
    const int64_t i = (int64_t)blockIdx.x * kBinThreads + threadIdx.x;
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
        qpart[2 * blockIdx.x] = s_q[0];
        qpart[2 * blockIdx.x + 1] = s_q2[0];
    }
}

constexpr int kScanThreads = 1024;

// One workgroup: exclusive scan of the cell counts into cell_start (ncell+1
// entries), then counts and fill are cleared for the next evaluation.  Also
// reduces the per-block charge sums into scalars[0] = Q, scalars[1] = sum q^2.
__global__ __launch_bounds__(kScanThreads) void k_scan(int ncell, int *__restrict__ counts,
                                                       int *__restrict__ fill, int *__restrict__ cell_start,
                                                       const double *__restrict__ qpart, int n_qblocks,
                                                       double *__restrict__ scalars, int *__restrict__ item_cell,
                                                       int *__restrict__ item_off, int *__restrict__ n_items)
{
    __shared__ int s_sum[kScanThreads];
    __shared__ int s_items[kScanThreads];
    __shared__ double s_a[kScanThreads];
    __shared__ double s_b[kScanThreads];
    const int t = threadIdx.x;
    const int per = (ncell + kScanThreads - 1) / kScanThreads;
    const int lo = t * per < ncell ? t * per : ncell;
    const int hi = lo + per < ncell ? lo + per : ncell;
    // pair-loop work items: one per (cell, kPairHome home particles)
    int local = 0, litems = 0;
    for (int c = lo; c < hi; ++c) {
        const int k = counts[c];
        local += k;
        litems += (k + kPairHome - 1) / kPairHome;
    }
    s_sum[t] = local;
    s_items[t] = litems;
    __syncthreads();
    // Hillis-Steele inclusive scans over the per-thread sums
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int v = t >= off ? s_sum[t - off] : 0;
        const int w = t >= off ? s_items[t - off] : 0;
        __syncthreads();
        s_sum[t] += v;
        s_items[t] += w;
        __syncthreads();
    }
    int run = s_sum[t] - local;
    int irun = s_items[t] - litems;
    for (int c = lo; c < hi; ++c) {
        const int k = counts[c];
        cell_start[c] = run;
        run += k;
        for (int o = 0; o < k; o += kPairHome) {
            item_cell[irun] = c;
            item_off[irun] = o;
            ++irun;
        }
        counts[c] = 0;
        fill[c] = 0;
    }
    if (t == kScanThreads - 1) {
        cell_start[ncell] = s_sum[t];
        *n_items = s_items[t];
    }

    // charge sums in a fixed order: contiguous ranges, then a fixed tree
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

__global__ __launch_bounds__(256) void k_scatter(int64_t n, const int *__restrict__ cell_of,
                                                 const int *__restrict__ cell_start, int *__restrict__ fill,
                                                 int *__restrict__ tmp_idx)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int c = cell_of[i];
    const int slot = cell_start[c] + atomicAdd(&fill[c], 1);
    tmp_idx[slot] = (int)i;
}

constexpr int kSortThreads = 128;
constexpr int kSortLds = 2048;

// One workgroup per cell.  The scatter above claimed slots in arbitrary order;
// the rank of an entry is the number of entries of the same cell with a smaller
// input index, so writing to cell_start + rank restores input order.
__global__ __launch_bounds__(kSortThreads) void k_cellsort(double L, const int *__restrict__ cell_start,
                                                           const int *__restrict__ tmp_idx,
                                                           const double *__restrict__ pos,
                                                           const double *__restrict__ q, int *__restrict__ perm,
                                                           d4 *__restrict__ pq)
{
    __shared__ int s_idx[kSortLds];
    const int c = blockIdx.x;
    const int start = cell_start[c];
    const int cnt = cell_start[c + 1] - start;
    const bool in_lds = cnt <= kSortLds;
    if (in_lds) {
        for (int e = threadIdx.x; e < cnt; e += kSortThreads) s_idx[e] = tmp_idx[start + e];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < cnt; e += kSortThreads) {
        const int mine = in_lds ? s_idx[e] : tmp_idx[start + e];
        int rank = 0;
        if (in_lds) {
            for (int f = 0; f < cnt; ++f) rank += s_idx[f] < mine;
        } else {
            for (int f = 0; f < cnt; ++f) rank += tmp_idx[start + f] < mine;
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

// Clears `words` 16-byte words (the counters and padding an evaluation expects
// at zero, when its buffers come from memory another evaluation used).
__global__ __launch_bounds__(256) void k_zero(uint4 *__restrict__ p, int64_t words)
{
    const uint4 z = {0u, 0u, 0u, 0u};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (int64_t)gridDim.x * 256) p[i] = z;
}

}  // namespace

hipError_t launch_zero(hipStream_t s, void *p, size_t bytes)
{
    const int64_t words = (int64_t)(bytes / sizeof(uint4));
    if (words == 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>(ceil_div(words, 256), 2048);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, static_cast<uint4 *>(p), words);
    return hipGetLastError();
}

hipError_t launch_bin(hipStream_t s, const CellArgs &a, const double *pos, const double *q, int *cell_of,
                      int *counts, double *qpart, int *status)
{
    hipLaunchKernelGGL(k_bin, dim3(ceil_div(a.n, kBinThreads)), dim3(kBinThreads), 0, s, a.n, a.L, a.nc, pos,
                       q, cell_of, counts, qpart, status);
    return hipGetLastError();
}

hipError_t launch_scan(hipStream_t s, const CellArgs &a, int *counts, int *fill, int *cell_start,
                       const double *qpart, int n_qblocks, double *scalars, int *item_cell, int *item_off,
                       int *n_items)
{
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, s, a.ncell, counts, fill, cell_start, qpart,
                       n_qblocks, scalars, item_cell, item_off, n_items);
    return hipGetLastError();
}

hipError_t launch_scatter(hipStream_t s, const CellArgs &a, const int *cell_of, const int *cell_start,
                          int *fill, int *tmp_idx)
{
    hipLaunchKernelGGL(k_scatter, dim3(ceil_div(a.n, 256)), dim3(256), 0, s, a.n, cell_of, cell_start, fill,
                       tmp_idx);
    return hipGetLastError();
}

hipError_t launch_cellsort(hipStream_t s, const CellArgs &a, const int *cell_start, const int *tmp_idx,
                           const double *pos, const double *q, int *perm, d4 *pq)
{
    hipLaunchKernelGGL(k_cellsort, dim3(a.ncell), dim3(kSortThreads), 0, s, a.L, cell_start, tmp_idx, pos, q,
                       perm, pq);
    return hipGetLastError();
}

int bin_blocks(int64_t n) { return ceil_div(n, kBinThreads); }

}  // namespace ewk
