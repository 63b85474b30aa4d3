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
//  1. k_pair_list: the non-empty neighbour ranges form one candidate stream,
//     taken 64 at a time (one candidate per lane, its range found from a bit
//     map of the range starts); the 8 home particles are wave-uniform.  For each home particle the in-range lanes are compacted
//     with a ballot and appended, in lane order, to that particle's list of
//     32-bit entries (sorted index | image-shift code << 25).
//  2. k_pair: 8 lanes per home particle (16 in mixed precision) walk its list
//     (lane s takes entries s, s+8, ...), so erfc/exp run only for pairs
//     inside r_c; the lanes' partial sums are combined by a fixed xor-shuffle
//     tree.
// Small systems, with too few work items to fill the chip, split an item's
// homes over up to 8 list waves and give each particle a whole wave (64
// lanes) in the evaluation pass.
// Both passes run in a fixed order, so results are bitwise reproducible.  A home
// particle whose list would overflow is evaluated by the exact direct loop
// instead.
//
// Precision: FP64 computes everything in double (erfc as exp(-x^2) times an FP64
// polynomial fit of erfc(x) exp(x^2) when sqrt(alpha) r_c <= 8, the library erfc
// otherwise).  MIXED forms d and |d|^2 in
// FP64 (exact cutoff test, no cancellation), evaluates the pair terms in FP32
// (erfc as exp(-x^2) times a polynomial fit of erfc(x) exp(x^2), the Gaussian
// from the FP64 exponent), and accumulates phi and F in FP64.
#include "ewald_internal.h"
#include "erfcx_fit.h"

namespace ewk {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kLog2e = 1.44269504088896340735992468100189214;

struct PairConsts {
    double sa, tsap, alpha, nal2;
    float saf, tsapf;
};

__device__ inline PairConsts pair_consts(double alpha)
{
    PairConsts k;
    k.alpha = alpha;
    k.sa = sqrt(alpha);
    k.tsap = 2.0 * sqrt(alpha / kPi);
    k.nal2 = -alpha * kLog2e;
    k.saf = (float)k.sa;
    k.tsapf = (float)k.tsap;
    return k;
}

// exp(-alpha r^2) in FP32 from the FP64 exponent: 2^a with a = -alpha log2(e) r^2
// split as n + f, n = rint(a), so the FP32 power of two sees |f| <= 1/2 and the
// exponent's own FP32 rounding does not grow with alpha r^2.
__device__ inline float gauss_f32(double r2, const PairConsts &k)
{
    const double a = k.nal2 * r2;
    const double n = __builtin_rint(a);
    return __builtin_amdgcn_ldexpf(__builtin_amdgcn_exp2f((float)(a - n)), (int)n);
}

// a b + c as one three-operand FP64 FMA.  Written out because the compiler
// otherwise turns a Horner step whose constant lives in a register into a copy
// of the constant followed by the accumulating two-operand form.
__device__ inline double fma3_f64(double a, double b, double c)
{
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

// Taylor coefficients ln(2)^k / k! of 2^f = e^(f ln 2).
constexpr double exp2_taylor(int k)
{
    double c = 1.0;
    for (int i = 1; i <= k; ++i) c = c * 0.69314718055994530941723212145817657 / (double)i;
    return c;
}

// exp(-alpha r^2) in FP64: 2^a with a = -alpha log2(e) r^2 split as n + f, n =
// rint(a), |f| <= 1/2, and 2^f by its Taylor series to degree 13 (truncation
// below 1e-17 relative), in three-operand FMAs.
__device__ inline double gauss_f64(double r2, const PairConsts &k)
{
    constexpr int kDeg = 13;
    const double a = k.nal2 * r2;
    const double n = __builtin_rint(a);
    const double f = a - n;
    double acc = exp2_taylor(kDeg);
#pragma unroll
    for (int i = kDeg - 1; i >= 0; --i) acc = fma3_f64(acc, f, exp2_taylor(i));
    return __builtin_amdgcn_ldexp(acc, (int)n);
}

// erfc(x) exp(x^2) for x >= 0 in FP32 (polynomial in t = 1 / (1 + x / 2),
// coefficients in erfcx_fit.h).
__device__ inline float erfcx_f32(float x)
{
    const float t = __builtin_amdgcn_rcpf(1.0f + kErfcxT * x);
    float acc = kErfcxP[kErfcxDegree];
#pragma unroll
    for (int i = kErfcxDegree - 1; i >= 0; --i) acc = __builtin_fmaf(acc, t, kErfcxP[i]);
    return acc * t;
}

// erfc(x) exp(x^2) for 0 <= x <= kErfcx64XMax in FP64 (polynomial in the centred
// u of t = 1 / (1 + x / 2), coefficients in erfcx_fit.h); 1/d by the hardware
// reciprocal and two Newton steps.
__device__ inline double erfcx_f64(double x)
{
    const double d = fma(0.5, x, 1.0);
    double t = __builtin_amdgcn_rcp(d);
    t = fma(t, fma(-d, t, 1.0), t);
    t = fma(t, fma(-d, t, 1.0), t);
    const double u = (t - kErfcx64C) * kErfcx64InvH;
    double acc = kErfcx64Q[kErfcx64Degree];
#pragma unroll
    for (int i = kErfcx64Degree - 1; i >= 0; --i) acc = fma3_f64(acc, u, kErfcx64Q[i]);
    return acc * t;
}

// One pair inside the cutoff: accumulate phi += q_j erfc(sa r)/r and
// F += q_j [erfc(sa r)/r + 2 sqrt(a/pi) exp(-a r^2)] / r^2 * d (q_i applied later).
// MIXED writes erfc(sa r) = exp(-a r^2) erfcx(sa r), so the one Gaussian serves
// both terms; so does FP64 when FIT64 (sqrt(a) r_c within the FP64 fit's range),
// with 1/r from the hardware reciprocal square root and two Newton steps.
template <bool MIXED, bool FIT64>
__device__ inline void pair_term(double dx, double dy, double dz, double r2, double qj, const PairConsts &k,
                                 double &ph, double &fx, double &fy, double &fz)
{
    if constexpr (MIXED) {
        const float r2f = (float)r2;
        const float ri = __builtin_amdgcn_rsqf(r2f);
        const float e = gauss_f32(r2, k);
        const float ec = e * erfcx_f32(k.saf * (r2f * ri)) * ri;
        const float gg = k.tsapf * e;
        const float qf = (float)qj;
        const double f = (double)(qf * (ec + gg) * (ri * ri));
        ph += (double)(qf * ec);
        fx += f * dx;
        fy += f * dy;
        fz += f * dz;
    } else if constexpr (FIT64) {
        double ri = __builtin_amdgcn_rsq(r2);
        ri = fma(0.5 * ri, fma(-r2 * ri, ri, 1.0), ri);
        ri = fma(0.5 * ri, fma(-r2 * ri, ri, 1.0), ri);
        const double e = gauss_f64(r2, k);
        const double ec = e * erfcx_f64(k.sa * (r2 * ri)) * ri;
        const double f = qj * (ec + k.tsap * e) * (ri * ri);
        ph += qj * ec;
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

// Stream positions covered by one start-bit map (the map is rebuilt for every
// further kStreamSeg candidates of a larger neighbourhood).
constexpr int kStreamSeg = 2048;

// SPLIT waves share a work item's kPairHome home particles (kPairHome / SPLIT
// each): small systems, whose items are too few to fill the chip, trade
// streaming the candidates SPLIT times for SPLIT times the waves.  A home
// particle's list does not depend on which wave builds it.
template <int SPLIT>
__device__ __forceinline__ void pair_list_body(int bx, int by, int nc, double L, double rc2, int max_items,
                                               const int *__restrict__ n_items, const int *__restrict__ item_cell,
                                               const int *__restrict__ item_off, const int *__restrict__ cell_start,
                                               const d4 *__restrict__ pq, uint32_t *__restrict__ list,
                                               int *__restrict__ list_cnt, int cap)
{
    // the non-empty neighbour ranges of the home cell, in offset order: start,
    // stream position (exclusive prefix of the lengths), image-shift code and
    // shift; and a bit map of the stream positions at which a range starts
    __shared__ int s_start[kStencil], s_pre[kStencil], s_code[kStencil];
    __shared__ double s_sx[kStencil], s_sy[kStencil], s_sz[kStencil];
    __shared__ uint64_t s_bits[kStreamSeg / 64];
    // neighbouring cells share one XCD's L2: remap over the actual item count
    // (known on the device only), so that padding blocks do not pile up on one XCD
    constexpr int HPW = kPairHome / SPLIT;  // home particles of this wave
    const int nit = *n_items;
    const int nwork = nit * SPLIT;
    const int per = (nwork + kXcds - 1) / kXcds;
    if ((int)bx >= per * kXcds) return;
    const int wk = xcd_remap(bx, nwork);
    if (wk >= nwork) return;
    const int it = wk / SPLIT, part = wk % SPLIT;
    (void)max_items;
    const int lane = (int)threadIdx.x;
    const int c = item_cell[it];
    const int cx = c / (nc * nc), cy = (c / nc) % nc, cz = c % nc;
    const int end = cell_start[c + 1];
    const int i0 = cell_start[c] + item_off[it] + part * HPW;
    if (i0 >= end) return;  // the item has no home particles for this wave
    const int nh = (end - i0) < HPW ? (end - i0) : HPW;  // wave-uniform
    // lane l takes offsets l and l + 64
    int st[2], len[2], code[2], wxyz[2][3];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int o = lane + u * kLanes;
        len[u] = 0;
        st[u] = 0;
        code[u] = 0;
        if (o < kStencil) {
            const int vx = wrap_count(cx + o / (kSpan * kSpan) - kPairReach, nc, wxyz[u][0]);
            const int vy = wrap_count(cy + (o / kSpan) % kSpan - kPairReach, nc, wxyz[u][1]);
            const int vz = wrap_count(cz + o % kSpan - kPairReach, nc, wxyz[u][2]);
            const int cn = (vx * nc + vy) * nc + vz;
            st[u] = cell_start[cn];
            len[u] = cell_start[cn + 1] - st[u];
            code[u] = ((wxyz[u][0] + kPairReach) * kSpan + (wxyz[u][1] + kPairReach)) * kSpan +
                      (wxyz[u][2] + kPairReach);
        }
    }
    // stream positions: inclusive scans of the two halves' lengths
    int in0 = len[0], in1 = len[1];
#pragma unroll
    for (int d = 1; d < kLanes; d <<= 1) {
        const int t0 = __shfl_up(in0, d), t1 = __shfl_up(in1, d);
        if (lane >= d) {
            in0 += t0;
            in1 += t1;
        }
    }
    const int tot0 = __builtin_amdgcn_readlane(in0, kLanes - 1);
    const int total = tot0 + __builtin_amdgcn_readlane(in1, kLanes - 1);  // wave-uniform
    const int pre[2] = {in0 - len[0], tot0 + in1 - len[1]};
    // ordinals of the non-empty ranges
    const uint64_t ne0 = __builtin_amdgcn_ballot_w64(len[0] > 0);
    const uint64_t ne1 = __builtin_amdgcn_ballot_w64(len[1] > 0);
    const int mb0 = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(ne0 >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)ne0, 0u));
    const int mb1 = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(ne1 >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)ne1, 0u));
    const int ordv[2] = {mb0, (int)__popcll(ne0) + mb1};
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        if (len[u] > 0) {
            const int k = ordv[u];
            s_start[k] = st[u];
            s_pre[k] = pre[u];
            s_code[k] = code[u];
            s_sx[k] = (double)wxyz[u][0] * L;
            s_sy[k] = (double)wxyz[u][1] * L;
            s_sz[k] = (double)wxyz[u][2] * L;
        }
    }
    // ordinal of the home cell's own range without shift (never empty: it
    // holds the home particles)
    const int self_ord = __builtin_amdgcn_readlane(ordv[kCenter / kLanes], kCenter % kLanes);
    double hx[HPW], hy[HPW], hz[HPW];
    int cnt[HPW];
#pragma unroll
    for (int h = 0; h < HPW; ++h) {
        const d4 p = pq[i0 + (h < nh ? h : 0)];
        hx[h] = p.a;
        hy[h] = p.b;
        hz[h] = p.c;
        cnt[h] = 0;
    }
    // One stream of candidates: the non-empty ranges in offset order, 64 at a
    // time (lane l takes position P0 + l).  Lane l's range is the last one
    // starting at or before its position: its ordinal is the number of range
    // starts in [0, P0 + l], minus one, read off the start-bit map.
    uint32_t *const list_item = list + (size_t)i0 * cap;  // rows of the item's home particles
    int base = 0;  // range starts before the current chunk
    for (int seg = 0; seg < total; seg += kStreamSeg) {
        __syncthreads();  // the previous segment's map is no longer read
        for (int w = lane; w < kStreamSeg / 64; w += kLanes) s_bits[w] = 0;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int r = pre[u] - seg;
            if (len[u] > 0 && r >= 0 && r < kStreamSeg)
                atomicOr(reinterpret_cast<unsigned *>(s_bits) + (r >> 5), 1u << (r & 31));
        }
        __syncthreads();
        const int seg_end = total - seg < kStreamSeg ? total : seg + kStreamSeg;
        for (int P0 = seg; P0 < seg_end; P0 += kLanes) {
            const uint64_t mv = s_bits[(P0 - seg) >> 6];
            // readfirstlane works on 32-bit ints: zero-extend each half
            const uint32_t m_lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)mv);
            const uint32_t m_hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(mv >> 32));
            const uint64_t m = ((uint64_t)m_hi << 32) | (uint64_t)m_lo;
            const int below = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            const int k = base + below + (int)((m >> lane) & 1u) - 1;
            base += __popcll(m);
            const int p = P0 + lane;
            const bool valid = p < total;
            const int j = valid ? s_start[k] + (p - s_pre[k]) : 0;
            const d4 q = pq[j];
            // lanes past the stream's end sit at an infinite distance (r2
            // overflows to +inf), so the cutoff test alone rejects them
            const double far = valid ? 0.0 : 1e300;
            const double px = q.a + s_sx[k] + far, py = q.b + s_sy[k], pz = q.c + s_sz[k];
            const uint32_t entry = (uint32_t)j | ((uint32_t)s_code[k] << kPairIndexBits);
            const int self = k == self_ord ? j : -1;  // the home cell without shift
#pragma unroll
            for (int h = 0; h < HPW; ++h) {
                if (h < nh) {
                    const double dx = hx[h] - px, dy = hy[h] - py, dz = hz[h] - pz;
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    const bool in = (r2 < rc2) & (self != i0 + h);
                    // the ballots of the two compares (lane masks as they stand),
                    // not of their combination, which would be rebuilt from a
                    // per-lane 0/1 value
                    const uint64_t mk =
                        __builtin_amdgcn_ballot_w64(r2 < rc2) & __builtin_amdgcn_ballot_w64(self != i0 + h);
                    if (mk != 0) {  // wave-uniform: most chunks hold no pair of most homes
                        int pos = cnt[h] + (int)__builtin_amdgcn_mbcnt_hi(
                                               (unsigned)(mk >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mk, 0u));
                        pos = pos < cap ? pos : cap - 1;  // an overflowing list is not used
                        // one uniform base for the item's rows plus an unsigned 32-bit offset
                        if (in) list_item[(unsigned)(h * cap) + (unsigned)pos] = entry;
                        cnt[h] += __popcll(mk);
                    }
                }
            }
        }
    }
    if (lane < nh) {
        int v = 0;
#pragma unroll
        for (int h = 0; h < HPW; ++h)
            if (h == lane) v = cnt[h];
        list_cnt[i0 + lane] = v > cap ? -1 : v;
    }
}

template <int SPLIT>
struct KPairList {
    static constexpr int kThreads = 64;
    static constexpr int kWavesPerEu = 1;
    int nc;
    double L;
    double rc2;
    int max_items;
    const int *n_items;
    const int *item_cell;
    const int *item_off;
    const int *cell_start;
    const d4 *pq;
    uint32_t *list;
    int *list_cnt;
    int cap;
    __device__ void run(int bx, int by) const
    {
        pair_list_body<SPLIT>(bx, by, nc, L, rc2, max_items, n_items, item_cell, item_off, cell_start, pq, list,
                              list_cnt, cap);
    }
    hipError_t one(hipStream_t s, dim3 grid, int threads, size_t smem) const;
};

template <int SPLIT>
__global__ __launch_bounds__(64) void k_pair_list(int nc, double L, double rc2, int max_items,
                                                  const int *__restrict__ n_items, const int *__restrict__ item_cell,
                                                  const int *__restrict__ item_off, const int *__restrict__ cell_start,
                                                  const d4 *__restrict__ pq, uint32_t *__restrict__ list,
                                                  int *__restrict__ list_cnt, int cap)
{
    pair_list_body<SPLIT>(blockIdx.x, blockIdx.y, nc, L, rc2, max_items, n_items, item_cell, item_off, cell_start, pq,
                          list, list_cnt, cap);
}

template <int SPLIT>
hipError_t KPairList<SPLIT>::one(hipStream_t s, dim3 grid, int threads, size_t smem) const
{
    hipLaunchKernelGGL((k_pair_list<SPLIT>), grid, dim3(threads), smem, s, nc, L, rc2, max_items, n_items, item_cell, item_off,
                       cell_start, pq, list, list_cnt, cap);
    return hipGetLastError();
}

// Evaluation pass: a work item is any HPW consecutive particles (lists carry
// global indices and image-shift codes, so no per-cell table is needed), each
// walked by 64 / HPW lanes: HPW = kPairHome (FP64), kPairHome / 2 (mixed), or 1
// for small systems, whose items are too few to fill the chip (the lanes of a
// particle, and so its sums, then differ; the choice depends on the precision
// and n alone).
template <bool MIXED, bool FIT64, int HPW>
__device__ __forceinline__ void pair_body(int bx, int by, int64_t n, int nc, double L, double rc2, double alpha,
                                          const int *__restrict__ cell_start, const d4 *__restrict__ pq,
                                          const uint32_t *__restrict__ list, const int *__restrict__ list_cnt, int cap,
                                          d4 *__restrict__ freal)
{
    constexpr int kSub = kLanes / HPW;  // lanes per home particle
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
    const int blocks = (int)((n + HPW - 1) / HPW);
    const int64_t i = (int64_t)xcd_remap(bx, blocks) * HPW + h;
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
        // mixed: keep the first entry's two loads here, in flight with the
        // others, rather than sunk into its predicated block (measured: the
        // kernel 65 against 66.5 us at 32^3, 476 against 493 us at 64^3; the
        // FP64 kernel gained nothing)
        if constexpr (MIXED) asm volatile("" ::"v"(p[0].a), "v"(p[0].b), "v"(p[0].c), "v"(p[0].d), "v"(e[0]));
        // FP64: entries without an image shift (every entry, in most waves) skip
        // the shift lookup; (x - 0) - y is x - y exactly, so results do not
        // change.  (In the mixed kernel the second copy of the loop cost more
        // registers than it saved: 3.5 % slower on a random k_max 40 system.)
        bool plain = !MIXED;
#pragma unroll
        for (int u = 0; u < kU; ++u)
            plain = plain && (r + u * kSub >= cnt_l || (int)(e[u] >> kPairIndexBits) == kCenter);
        if (!MIXED && __all(plain)) {
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                if (r + u * kSub < cnt_l) {
                    const double dx = me.a - p[u].a, dy = me.b - p[u].b, dz = me.c - p[u].c;
                    pair_term<MIXED, FIT64>(dx, dy, dz, dx * dx + dy * dy + dz * dz, p[u].d, k, ph, fx, fy, fz);
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                if (r + u * kSub < cnt_l) {
                    const int code = (int)(e[u] >> kPairIndexBits);
                    const double dx = (me.a - s_sh[code][0]) - p[u].a;
                    const double dy = (me.b - s_sh[code][1]) - p[u].b;
                    const double dz = (me.c - s_sh[code][2]) - p[u].c;
                    pair_term<MIXED, FIT64>(dx, dy, dz, dx * dx + dy * dy + dz * dz, p[u].d, k, ph, fx, fy, fz);
                }
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
                if (r2 < rc2 && !(o == kCenter && j == i)) pair_term<MIXED, FIT64>(dx, dy, dz, r2, p.d, k, ph, fx, fy, fz);
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

template <bool MIXED, bool FIT64, int HPW>
struct KPair {
    static constexpr int kThreads = 64;
    static constexpr int kWavesPerEu = 1;
    int64_t n;
    int nc;
    double L;
    double rc2;
    double alpha;
    const int *cell_start;
    const d4 *pq;
    const uint32_t *list;
    const int *list_cnt;
    int cap;
    d4 *freal;
    __device__ void run(int bx, int by) const
    {
        pair_body<MIXED, FIT64, HPW>(bx, by, n, nc, L, rc2, alpha, cell_start, pq, list, list_cnt, cap, freal);
    }
    hipError_t one(hipStream_t s, dim3 grid, int threads, size_t smem) const;
};

template <bool MIXED, bool FIT64, int HPW>
__global__ __launch_bounds__(64) void k_pair(int64_t n, int nc, double L, double rc2, double alpha,
                                             const int *__restrict__ cell_start, const d4 *__restrict__ pq,
                                             const uint32_t *__restrict__ list, const int *__restrict__ list_cnt,
                                             int cap, d4 *__restrict__ freal)
{
    pair_body<MIXED, FIT64, HPW>(blockIdx.x, blockIdx.y, n, nc, L, rc2, alpha, cell_start, pq, list, list_cnt, cap,
                                 freal);
}

template <bool MIXED, bool FIT64, int HPW>
hipError_t KPair<MIXED, FIT64, HPW>::one(hipStream_t s, dim3 grid, int threads, size_t smem) const
{
    hipLaunchKernelGGL((k_pair<MIXED, FIT64, HPW>), grid, dim3(threads), smem, s, n, nc, L, rc2, alpha, cell_start, pq, list,
                       list_cnt, cap, freal);
    return hipGetLastError();
}

}  // namespace

int pair_list_split(int max_items)
{
    int split = 1;
    while (split < kPairHome && (int64_t)max_items * split < kPairSmallWaves) split *= 2;
    return split;
}

bool pair_small(int64_t n) { return ceil_div(n, kPairHome) < kPairSmallWaves / 2; }

namespace {

template <int SPLIT>
hipError_t launch_list(hipStream_t s, const PairArgs &a, int max_items, const int *n_items, const int *item_cell,
                       const int *item_off, const int *cell_start, const d4 *pq, uint32_t *list, int *list_cnt, int cap)
{
    return launch(s, dim3(xcd_grid(max_items * SPLIT)), 64, 0,
                  KPairList<SPLIT>{a.nc, a.L, a.rc2, max_items, n_items, item_cell, item_off, cell_start, pq, list,
                                   list_cnt, cap});
}

template <int HPW>
hipError_t launch_eval(hipStream_t s, const PairArgs &a, bool mixed, const int *cell_start, const d4 *pq,
                       const uint32_t *list, const int *list_cnt, int cap, d4 *freal)
{
    const int blocks = xcd_grid(ceil_div(a.n, HPW));
    // the FP64 erfcx polynomial covers sqrt(alpha) r <= kErfcx64XMax
    const bool fit64 = sqrt(a.alpha * a.rc2) <= kErfcx64XMax;
    if (mixed)
        return launch(s, dim3(blocks), 64, 0,
                      KPair<true, false, HPW>{a.n, a.nc, a.L, a.rc2, a.alpha, cell_start, pq, list, list_cnt, cap,
                                              freal});
    if (fit64)
        return launch(s, dim3(blocks), 64, 0,
                      KPair<false, true, HPW>{a.n, a.nc, a.L, a.rc2, a.alpha, cell_start, pq, list, list_cnt, cap,
                                              freal});
    return launch(s, dim3(blocks), 64, 0,
                  KPair<false, false, HPW>{a.n, a.nc, a.L, a.rc2, a.alpha, cell_start, pq, list, list_cnt, cap,
                                           freal});
}

}  // namespace

hipError_t launch_pair_list(hipStream_t s, const PairArgs &a, int max_items, const int *n_items,
                            const int *item_cell, const int *item_off, const int *cell_start, const d4 *pq,
                            uint32_t *list, int *list_cnt, int cap)
{
    switch (pair_list_split(max_items)) {
    case 1: return launch_list<1>(s, a, max_items, n_items, item_cell, item_off, cell_start, pq, list, list_cnt, cap);
    case 2: return launch_list<2>(s, a, max_items, n_items, item_cell, item_off, cell_start, pq, list, list_cnt, cap);
    case 4: return launch_list<4>(s, a, max_items, n_items, item_cell, item_off, cell_start, pq, list, list_cnt, cap);
    default:
        return launch_list<8>(s, a, max_items, n_items, item_cell, item_off, cell_start, pq, list, list_cnt, cap);
    }
}

hipError_t launch_pair(hipStream_t s, const PairArgs &a, bool mixed, const int *cell_start, const d4 *pq,
                       const uint32_t *list, const int *list_cnt, int cap, d4 *freal)
{
    if (pair_small(a.n)) return launch_eval<1>(s, a, mixed, cell_start, pq, list, list_cnt, cap, freal);
    // the mixed kernel (70 VGPRs) takes twice the waves of kPairHome particles
    // each, to hide its load latency: 0.198 against 0.204 ms per 32^3
    // evaluation; the FP64 one (160 VGPRs) is already at its occupancy limit
    if (mixed) return launch_eval<kPairHome / 2>(s, a, mixed, cell_start, pq, list, list_cnt, cap, freal);
    return launch_eval<kPairHome>(s, a, mixed, cell_start, pq, list, list_cnt, cap, freal);
}

}  // namespace ewk
