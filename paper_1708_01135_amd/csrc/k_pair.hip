// Real-space part of the Ewald sum (section 3.2.1, Eq. short_range_force):
//
//   phi_i = sum_{(j,s) != (i,0), |d| < r_c} q_j erfc(sqrt(alpha)|d|)/|d|,   d = r_i - r_j - s
//   F_i   = q_i sum (same set) q_j d/|d|^2 [erfc(sqrt(alpha)|d|)/|d| + 2 sqrt(alpha/pi) exp(-alpha|d|^2)]
//
// Every ordered pair is visited from its i side and forces are written to i
// alone (as in the paper's pair kernel), so there are no write conflicts and no
// atomics.  Cells have side h = L/nc >= r_c; the 27 neighbours of a cell are
// taken as unwrapped offsets, each naming one (cell, image shift) pair, which
// stays exact for nc = 1 or 2 where one cell appears under several shifts.
//
// Work item = up to kPairHome (8) home particles of one cell; two passes:
//  1. k_pair_list: lanes hold 64 candidates at a time (one z-column of three
//     neighbour cells, read coalesced), the 8 home particles are wave-uniform.
//     For each home particle the in-range lanes are compacted with a ballot and
//     appended, in lane order, to that particle's list of 16-bit entries
//     (neighbour offset code << 11 | index inside that neighbour cell).
//  2. k_pair: 8 lanes per home particle walk its list (lane s takes entries
//     s, s+8, ...), so erfc/exp run only for pairs inside r_c; the 8 partial
//     sums are combined by a fixed xor-shuffle tree.
// Both passes run in a fixed order, so results are bitwise reproducible.  A home
// particle whose list would overflow, or whose neighbourhood holds a cell of
// more than 2048 particles, is evaluated by the exact direct loop instead.
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

// Neighbour o = (ox+1)*9 + (oy+1)*3 + (oz+1) of cell (cx, cy, cz): wrapped cell
// id and the image shift s that is added to the neighbour's positions.
__device__ inline int neighbour(int nc, double L, int cx, int cy, int cz, int o, double &sx, double &sy,
                                double &sz)
{
    int vx = cx + o / 9 - 1, vy = cy + (o / 3) % 3 - 1, vz = cz + o % 3 - 1;
    sx = sy = sz = 0.0;
    if (vx < 0) { vx += nc; sx = -L; } else if (vx >= nc) { vx -= nc; sx = L; }
    if (vy < 0) { vy += nc; sy = -L; } else if (vy >= nc) { vy -= nc; sy = L; }
    if (vz < 0) { vz += nc; sz = -L; } else if (vz >= nc) { vz -= nc; sz = L; }
    return (vx * nc + vy) * nc + vz;
}

constexpr int kCenter = 13;  // offset code of the home cell itself (zero shift)

__global__ __launch_bounds__(64) void k_pair_list(int nc, double L, double rc2, const int *__restrict__ n_items,
                                                  const int *__restrict__ item_cell, const int *__restrict__ item_off,
                                                  const int *__restrict__ cell_start, const d4 *__restrict__ pq,
                                                  uint16_t *__restrict__ list, int *__restrict__ list_cnt, int cap)
{
    const int it = blockIdx.x;
    if (it >= *n_items) return;
    const int lane = (int)threadIdx.x;
    const int c = item_cell[it];
    const int cx = c / (nc * nc), cy = (c / nc) % nc, cz = c % nc;
    const int end = cell_start[c + 1];
    const int i0 = cell_start[c] + item_off[it];
    const int nh = (end - i0) < kPairHome ? (end - i0) : kPairHome;  // wave-uniform
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
    bool big = false;
    for (int col = 0; col < 9; ++col) {
        // the three cells of neighbour column col, as up to three ranges
        int rs[3], rl[3], ro[3];
        double rsx[3], rsy[3], rsz[3];
        int tot = 0;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int o = col * 3 + t;
            const int cn = neighbour(nc, L, cx, cy, cz, o, rsx[t], rsy[t], rsz[t]);
            rs[t] = cell_start[cn];
            rl[t] = cell_start[cn + 1] - rs[t];
            ro[t] = o;
            if (rl[t] > kPairMaxCell) {
                big = true;
                rl[t] = 0;
            }
            tot += rl[t];
        }
        for (int p0 = 0; p0 < tot; p0 += kLanes) {
            const int p = p0 + lane;
            const bool valid = p < tot;
            const int t = p < rl[0] ? 0 : (p < rl[0] + rl[1] ? 1 : 2);
            const int local = p - (t == 0 ? 0 : (t == 1 ? rl[0] : rl[0] + rl[1]));
            const int j = (t == 0 ? rs[0] : (t == 1 ? rs[1] : rs[2])) + (valid ? local : 0);
            const int o = t == 0 ? ro[0] : (t == 1 ? ro[1] : ro[2]);
            const d4 q = pq[valid ? j : 0];
            const double px = q.a + (t == 0 ? rsx[0] : (t == 1 ? rsx[1] : rsx[2]));
            const double py = q.b + (t == 0 ? rsy[0] : (t == 1 ? rsy[1] : rsy[2]));
            const double pz = q.c + (t == 0 ? rsz[0] : (t == 1 ? rsz[1] : rsz[2]));
            const uint16_t entry = (uint16_t)((o << kPairLocalBits) | (valid ? local : 0));
#pragma unroll
            for (int h = 0; h < kPairHome; ++h) {
                if (h < nh) {
                    const double dx = hx[h] - px, dy = hy[h] - py, dz = hz[h] - pz;
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    const bool in = valid && r2 < rc2 && !(o == kCenter && j == i0 + h);
                    const uint64_t m = __ballot(in);
                    const int pos = cnt[h] + (int)__builtin_amdgcn_mbcnt_hi(
                                                 (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
                    if (in && pos < cap) list[(size_t)(i0 + h) * cap + pos] = entry;
                    cnt[h] += __popcll(m);
                }
            }
        }
    }
    if (lane < nh) {
        int v = 0;
#pragma unroll
        for (int h = 0; h < kPairHome; ++h)
            if (h == lane) v = cnt[h];
        list_cnt[i0 + lane] = (big || v > cap) ? -1 : v;
    }
}

template <bool MIXED>
__global__ __launch_bounds__(64) void k_pair(int nc, double L, double rc2, double alpha,
                                             const int *__restrict__ n_items, const int *__restrict__ item_cell,
                                             const int *__restrict__ item_off, const int *__restrict__ cell_start,
                                             const d4 *__restrict__ pq, const uint16_t *__restrict__ list,
                                             const int *__restrict__ list_cnt, int cap, d4 *__restrict__ freal)
{
    constexpr int kSub = kLanes / kPairHome;  // lanes per home particle
    __shared__ int s_js[27];
    __shared__ double s_sx[27], s_sy[27], s_sz[27];
    const int it = blockIdx.x;
    if (it >= *n_items) return;
    const PairConsts k = pair_consts(alpha);
    const int c = item_cell[it];
    const int cx = c / (nc * nc), cy = (c / nc) % nc, cz = c % nc;
    const int end = cell_start[c + 1];
    const int lane = (int)threadIdx.x;
    const int h = lane / kSub, s = lane % kSub;
    const int i = cell_start[c] + item_off[it] + h;
    const bool act = i < end;
    if (lane < 27) {
        double sx, sy, sz;
        const int cn = neighbour(nc, L, cx, cy, cz, lane, sx, sy, sz);
        s_js[lane] = cell_start[cn];
        s_sx[lane] = sx;
        s_sy[lane] = sy;
        s_sz[lane] = sz;
    }
    __syncthreads();
    const d4 me = pq[act ? i : 0];
    const int cnt = act ? list_cnt[i] : 0;
    double ph = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    const uint16_t *mine = list + (size_t)(act ? i : 0) * cap;
    for (int r = s; __any(r < cnt); r += kSub) {
        if (r < cnt) {
            const unsigned e = mine[r];
            const int o = (int)(e >> kPairLocalBits);
            const d4 p = pq[s_js[o] + (int)(e & (kPairMaxCell - 1))];
            const double dx = (me.a - s_sx[o]) - p.a;
            const double dy = (me.b - s_sy[o]) - p.b;
            const double dz = (me.c - s_sz[o]) - p.c;
            pair_term<MIXED>(dx, dy, dz, dx * dx + dy * dy + dz * dz, p.d, k, ph, fx, fy, fz);
        }
    }
    if (__any(cnt < 0)) {
        // exact direct loop for particles whose list overflowed; sub-lane s
        // takes the neighbour offsets o = s, s + kSub, ...
        const bool slow = cnt < 0;
        for (int o = s; o < 27; o += kSub) {
            double sx, sy, sz;
            const int cn = neighbour(nc, L, cx, cy, cz, o, sx, sy, sz);
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
                            uint16_t *list, int *list_cnt, int cap)
{
    hipLaunchKernelGGL(k_pair_list, dim3(max_items), dim3(64), 0, s, a.nc, a.L, a.rc2, n_items, item_cell, item_off,
                       cell_start, pq, list, list_cnt, cap);
    return hipGetLastError();
}

hipError_t launch_pair(hipStream_t s, const PairArgs &a, bool mixed, int max_items, const int *n_items,
                       const int *item_cell, const int *item_off, const int *cell_start, const d4 *pq,
                       const uint16_t *list, const int *list_cnt, int cap, d4 *freal)
{
    if (mixed)
        hipLaunchKernelGGL(k_pair<true>, dim3(max_items), dim3(64), 0, s, a.nc, a.L, a.rc2, a.alpha, n_items,
                           item_cell, item_off, cell_start, pq, list, list_cnt, cap, freal);
    else
        hipLaunchKernelGGL(k_pair<false>, dim3(max_items), dim3(64), 0, s, a.nc, a.L, a.rc2, a.alpha, n_items,
                           item_cell, item_off, cell_start, pq, list, list_cnt, cap, freal);
    return hipGetLastError();
}

}  // namespace ewk
