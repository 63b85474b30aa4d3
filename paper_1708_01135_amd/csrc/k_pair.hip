// Real-space part of the Ewald sum (section 3.2.1, Eq. short_range_force):
//
//   phi_i = sum_{(j,s) != (i,0), |d| < r_c} q_j erfc(sqrt(alpha)|d|)/|d|,   d = r_i - r_j - s
//   F_i   = q_i sum (same set) q_j d/|d|^2 [erfc(sqrt(alpha)|d|)/|d| + 2 sqrt(alpha/pi) exp(-alpha|d|^2)]
//
// Every ordered pair is visited from its i side and forces are written to i
// alone (as in the paper's pair kernel), so there are no write conflicts and no
// atomics.  Cells have side h = L/nc >= r_c/2, so every image within r_c lies in
// the 5^3 cells around a particle's own; the neighbours are taken as unwrapped
// offsets, each naming one (cell, image shift) pair, which stays exact for small
// nc where one cell appears under several shifts.
//
// Work item = up to kPairHome (8) home particles of one cell; two passes:
//  1. k_pair_list: the 125 neighbour ranges form one candidate stream, taken
//     64 at a time (one candidate per lane); the 8 home particles are
//     wave-uniform.  For each home particle the in-range lanes are compacted
//     with a ballot and appended, in lane order, to that particle's list of
//     32-bit entries (sorted index | image-shift code << 25).
//  2. k_pair: 8 lanes per home particle walk its list (lane s takes entries
//     s, s+8, ...), so erfc/exp run only for pairs inside r_c; the 8 partial
//     sums are combined by a fixed xor-shuffle tree.
// Both passes run in a fixed order, so results are bitwise reproducible.  A home
// particle whose list would overflow, or whose neighbourhood holds a cell of
// more than 512 particles, is evaluated by the exact direct loop instead.
//
// Precision: FP64 computes everything in double.  MIXED forms d and |d|^2 in
// FP64 (exact cutoff test, no cancellation), evaluates erfc/exp/rsqrt in FP32,
// and accumulates phi and F in FP64.
#include "ewald_internal.h"

namespace ewk {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

struct PairConsts {
    double sa, tsap, alpha;
    float saf, tsapf, alphaf;
};

__device__ inline PairConsts pair_consts(double alpha)
{
    PairConsts k;
    k.alpha = alpha;
    k.sa = sqrt(alpha);
    k.tsap = 2.0 * sqrt(alpha / kPi);
    k.saf = (float)k.sa;
    k.tsapf = (float)k.tsap;
    k.alphaf = (float)alpha;
    return k;
}

// One pair inside the cutoff: accumulate phi += q_j erfc(sa r)/r and
// F += q_j [erfc(sa r)/r + 2 sqrt(a/pi) exp(-a r^2)] / r^2 * d (q_i applied later).
template <bool MIXED>
__device__ inline void pair_term(double dx, double dy, double dz, double r2, double qj, const PairConsts &k,
                                 double &ph, double &fx, double &fy, double &fz)
{
    if constexpr (MIXED) {
        const float r2f = (float)r2;
        const float ri = rsqrtf(r2f);
        const float ec = erfcf(k.saf * (r2f * ri)) * ri;
        const float gg = k.tsapf * expf(-k.alphaf * r2f);
        const float qf = (float)qj;
        const double f = (double)(qf * (ec + gg) * (ri * ri));
        ph += (double)(qf * ec);
        fx += f * dx;
        fy += f * dy;
        fz += f * dz;
    } else {
        const double r = sqrt(r2);
        const double ec = erfc(k.sa * r) / r;
        const double f = qj * (ec + k.tsap * exp(-k.alpha * r2)) / r2;
        ph += qj * ec;
        fx += f * dx;
        fy += f * dy;
        fz += f * dz;
    }
}

constexpr int kSpan = 2 * kPairReach + 1;              // cells per axis in the stencil
constexpr int kStencil = kSpan * kSpan * kSpan;          // neighbour offsets
constexpr int kCenter = (kStencil - 1) / 2;              // the home cell itself (zero shift)

// Neighbour o = ((ox+R)*kSpan + (oy+R))*kSpan + (oz+R) of cell (cx, cy, cz), R =
// kPairReach: wrapped cell id and the image shift s added to its positions.
__device__ inline int wrap_axis(int v, int nc, double L, double &sh)
{
    int w = v >= 0 ? v / nc : -((-v + nc - 1) / nc);  // floor(v / nc)
    sh = (double)w * L;
    return v - w * nc;
}

__device__ inline int neighbour(int nc, double L, int cx, int cy, int cz, int o, double &sx, double &sy,
                                double &sz)
{
    const int vx = wrap_axis(cx + o / (kSpan * kSpan) - kPairReach, nc, L, sx);
    const int vy = wrap_axis(cy + (o / kSpan) % kSpan - kPairReach, nc, L, sy);
    const int vz = wrap_axis(cz + o % kSpan - kPairReach, nc, L, sz);
    return (vx * nc + vy) * nc + vz;
}


// Cell index and wrap count along one axis: v = w nc + cell, w = floor(v / nc).
__device__ inline int wrap_count(int v, int nc, int &w)
{
    w = v >= 0 ? v / nc : -((-v + nc - 1) / nc);
    return v - w * nc;
}

__global__ __launch_bounds__(64) void k_pair_list(int nc, double L, double rc2, int max_items,
                                                  const int *__restrict__ n_items,
                                                  const int *__restrict__ item_cell, const int *__restrict__ item_off,
                                                  const int *__restrict__ cell_start, const d4 *__restrict__ pq,
                                                  uint32_t *__restrict__ list, int *__restrict__ list_cnt, int cap)
{
    // neighbour ranges of the home cell: start, length, image shift and code,
    // and the exclusive prefix of the lengths (the candidate stream position of
    // each neighbour range)
    __shared__ int s_start[kStencil], s_len[kStencil], s_code[kStencil], s_pre[kStencil];
    __shared__ double s_sx[kStencil], s_sy[kStencil], s_sz[kStencil];
    // neighbouring cells share one XCD's L2: remap over the actual item count
    // (known on the device only), so that padding blocks do not pile up on one XCD
    const int nit = *n_items;
    const int per = (nit + kXcds - 1) / kXcds;
    if ((int)blockIdx.x >= per * kXcds) return;
    const int it = xcd_remap(blockIdx.x, nit);
    if (it >= nit) return;
    (void)max_items;
    const int lane = (int)threadIdx.x;
    const int c = item_cell[it];
    const int cx = c / (nc * nc), cy = (c / nc) % nc, cz = c % nc;
    const int end = cell_start[c + 1];
    const int i0 = cell_start[c] + item_off[it];
    const int nh = (end - i0) < kPairHome ? (end - i0) : kPairHome;  // wave-uniform
    for (int o = lane; o < kStencil; o += kLanes) {
        int wx, wy, wz;
        const int vx = wrap_count(cx + o / (kSpan * kSpan) - kPairReach, nc, wx);
        const int vy = wrap_count(cy + (o / kSpan) % kSpan - kPairReach, nc, wy);
        const int vz = wrap_count(cz + o % kSpan - kPairReach, nc, wz);
        const int cn = (vx * nc + vy) * nc + vz;
        s_start[o] = cell_start[cn];
        s_len[o] = cell_start[cn + 1] - s_start[o];
        s_code[o] = ((wx + kPairReach) * kSpan + (wy + kPairReach)) * kSpan + (wz + kPairReach);
        s_sx[o] = (double)wx * L;
        s_sy[o] = (double)wy * L;
        s_sz[o] = (double)wz * L;
    }
    double hx[kPairHome], hy[kPairHome], hz[kPairHome];
    int cnt[kPairHome];
#pragma unroll
    for (int h = 0; h < kPairHome; ++h) {
        const d4 p = pq[i0 + (h < nh ? h : 0)];
        hx[h] = p.a;
        hy[h] = p.b;
        hz[h] = p.c;
        cnt[h] = 0;
    }
    __syncthreads();
    // exclusive prefix of the 125 lengths; lane l keeps those of offsets l and
    // l + 64 in registers (read back wave-uniformly with readlane)
    const int l0 = lane < kStencil ? s_len[lane] : 0;
    const int l1 = lane + kLanes < kStencil ? s_len[lane + kLanes] : 0;
    int in0 = l0, in1 = l1;
#pragma unroll
    for (int d = 1; d < kLanes; d <<= 1) {
        const int t0 = __shfl_up(in0, d), t1 = __shfl_up(in1, d);
        if (lane >= d) {
            in0 += t0;
            in1 += t1;
        }
    }
    const int tot0 = __shfl(in0, kLanes - 1);
    const int pre_lo = in0 - l0, pre_hi = tot0 + in1 - l1;
    const int total = tot0 + __shfl(in1, kLanes - 1);
    if (lane < kStencil) s_pre[lane] = pre_lo;
    if (lane + kLanes < kStencil) s_pre[lane + kLanes] = pre_hi;
    __syncthreads();
    // One stream of candidates: the neighbour ranges in offset order, 64 at a
    // time.  Lane l takes candidate P0 + l, in the last offset whose prefix is
    // <= P0 + l; the offsets that start inside the chunk are walked once per
    // chunk (wave-uniform), starting from the offset that held the previous
    // chunk's last candidate.
    int cur = 0;
    for (int P0 = 0; P0 < total; P0 += kLanes) {
        const int p = P0 + lane;
        const bool valid = p < total;
        int o = cur;
        for (int k = cur + 1; k < kStencil; ++k) {
            const int pk = k < kLanes ? __builtin_amdgcn_readlane(pre_lo, k) : __builtin_amdgcn_readlane(pre_hi, k - kLanes);
            if (pk >= P0 + kLanes) break;
            o += p >= pk ? 1 : 0;
        }
        cur = __builtin_amdgcn_readlane(o, kLanes - 1);
        const int j = valid ? s_start[o] + (p - s_pre[o]) : 0;
        const d4 q = pq[j];
        const double px = q.a + s_sx[o], py = q.b + s_sy[o], pz = q.c + s_sz[o];
        const uint32_t entry = (uint32_t)j | ((uint32_t)s_code[o] << kPairIndexBits);
        const int self = (valid && o == kCenter) ? j : -1;  // the home cell without shift
#pragma unroll
        for (int h = 0; h < kPairHome; ++h) {
            if (h < nh) {
                const double dx = hx[h] - px, dy = hy[h] - py, dz = hz[h] - pz;
                const double r2 = dx * dx + dy * dy + dz * dz;
                const bool in = valid && r2 < rc2 && self != i0 + h;
                const uint64_t m = __ballot(in);
                int pos = cnt[h] + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
                pos = pos < cap ? pos : cap - 1;  // an overflowing list is not used
                if (in) list[(size_t)(i0 + h) * cap + pos] = entry;
                cnt[h] += __popcll(m);
            }
        }
    }
    if (lane < nh) {
        int v = 0;
#pragma unroll
        for (int h = 0; h < kPairHome; ++h)
            if (h == lane) v = cnt[h];
        list_cnt[i0 + lane] = v > cap ? -1 : v;
    }
}

// Evaluation pass: a work item is any kPairHome consecutive particles (lists
// carry global indices and image-shift codes, so no per-cell table is needed).
template <bool MIXED>
__global__ __launch_bounds__(64) void k_pair(int64_t n, int nc, double L, double rc2, double alpha,
                                             const int *__restrict__ cell_start, const d4 *__restrict__ pq,
                                             const uint32_t *__restrict__ list, const int *__restrict__ list_cnt,
                                             int cap, d4 *__restrict__ freal)
{
    constexpr int kSub = kLanes / kPairHome;  // lanes per home particle
    __shared__ double s_sh[kStencil][3];
    const PairConsts k = pair_consts(alpha);
    const int lane = (int)threadIdx.x;
    for (int code = lane; code < kStencil; code += kLanes) {
        s_sh[code][0] = (double)(code / (kSpan * kSpan) - kPairReach) * L;
        s_sh[code][1] = (double)((code / kSpan) % kSpan - kPairReach) * L;
        s_sh[code][2] = (double)(code % kSpan - kPairReach) * L;
    }
    __syncthreads();
    const int h = lane / kSub, s = lane % kSub;
    const int blocks = (int)((n + kPairHome - 1) / kPairHome);
    const int64_t i = (int64_t)xcd_remap(blockIdx.x, blocks) * kPairHome + h;
    const bool act = i < n;
    const d4 me = pq[act ? i : 0];
    const int cnt = act ? list_cnt[i] : 0;
    double ph = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    const uint32_t *mine = list + (size_t)(act ? i : 0) * cap;
    // four entries per step: the four list loads, then the four particle loads,
    // are in flight together (indices clamped inside this particle's list;
    // entries past the count are loaded but not used)
    constexpr int kU = 4;
    const int cnt_l = cnt > 0 ? cnt : 0;
    for (int r = s; __any(r < cnt_l); r += kU * kSub) {
        uint32_t e[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int rr = r + u * kSub;
            e[u] = mine[rr < cap ? rr : cap - 1];
        }
        d4 p[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const bool ok = r + u * kSub < cnt_l;
            p[u] = pq[ok ? (e[u] & ((1u << kPairIndexBits) - 1)) : 0];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            if (r + u * kSub < cnt_l) {
                const int code = (int)(e[u] >> kPairIndexBits);
                const double dx = (me.a - s_sh[code][0]) - p[u].a;
                const double dy = (me.b - s_sh[code][1]) - p[u].b;
                const double dz = (me.c - s_sh[code][2]) - p[u].c;
                pair_term<MIXED>(dx, dy, dz, dx * dx + dy * dy + dz * dz, p[u].d, k, ph, fx, fy, fz);
            }
        }
    }
    if (__any(cnt < 0)) {
        // exact direct loop for particles whose list overflowed; sub-lane s takes
        // the neighbour offsets o = s, s + kSub, ...
        const bool slow = cnt < 0;
        const int cx = (int)(me.a * nc / L), cy = (int)(me.b * nc / L), cz = (int)(me.c * nc / L);
        const int hx = cx < nc ? cx : nc - 1, hy = cy < nc ? cy : nc - 1, hz = cz < nc ? cz : nc - 1;
        for (int o = s; o < kStencil; o += kSub) {
            double sx, sy, sz;
            const int cn = neighbour(nc, L, hx, hy, hz, o, sx, sy, sz);
            const double xi = me.a - sx, yi = me.b - sy, zi = me.c - sz;
            const int js = cell_start[cn], je = cell_start[cn + 1];
            for (int j = js; slow && j < je; ++j) {
                const d4 p = pq[j];
                const double dx = xi - p.a, dy = yi - p.b, dz = zi - p.c;
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 < rc2 && !(o == kCenter && j == i)) pair_term<MIXED>(dx, dy, dz, r2, p.d, k, ph, fx, fy, fz);
            }
        }
    }
    // fixed-order tree over the kSub lanes of each home particle
#pragma unroll
    for (int w = 1; w < kSub; w <<= 1) {
        ph += __shfl_xor(ph, w);
        fx += __shfl_xor(fx, w);
        fy += __shfl_xor(fy, w);
        fz += __shfl_xor(fz, w);
    }
    if (act && s == 0) {
        d4 out;
        out.a = ph;
        out.b = me.d * fx;
        out.c = me.d * fy;
        out.d = me.d * fz;
        freal[i] = out;
    }
}

}  // namespace

hipError_t launch_pair_list(hipStream_t s, const PairArgs &a, int max_items, const int *n_items,
                            const int *item_cell, const int *item_off, const int *cell_start, const d4 *pq,
                            uint32_t *list, int *list_cnt, int cap)
{
    hipLaunchKernelGGL(k_pair_list, dim3(xcd_grid(max_items)), dim3(64), 0, s, a.nc, a.L, a.rc2, max_items, n_items,
                       item_cell, item_off, cell_start, pq, list, list_cnt, cap);
    return hipGetLastError();
}

hipError_t launch_pair(hipStream_t s, const PairArgs &a, bool mixed, const int *cell_start, const d4 *pq,
                       const uint32_t *list, const int *list_cnt, int cap, d4 *freal)
{
    const int blocks = xcd_grid(ceil_div(a.n, kPairHome));
    if (mixed)
        hipLaunchKernelGGL(k_pair<true>, dim3(blocks), dim3(64), 0, s, a.n, a.nc, a.L, a.rc2, a.alpha, cell_start, pq,
                           list, list_cnt, cap, freal);
    else
        hipLaunchKernelGGL(k_pair<false>, dim3(blocks), dim3(64), 0, s, a.n, a.nc, a.L, a.rc2, a.alpha, cell_start, pq,
                           list, list_cnt, cap, freal);
    return hipGetLastError();
}

}  // namespace ewk
