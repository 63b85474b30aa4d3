// Reciprocal-space part of the Ewald sum (section 3.1.2 and Eq. perf_mod1):
//
//   S_k = sum_j q_j exp(i k.r_j)                       (Algorithm 1, conjugated)
//   E_recip = sum_{k in K+} C_k |S_k|^2,  G_k = 2 C_k S_k
//   F_i = q_i (2 pi / L) sum_{k in K+} n Im(exp(i k.r_i) conj(G_k))   (Algorithm 2)
//   phi_i = sum_{k in K+} Re(exp(i k.r_i) conj(G_k))
//
// K+ is the half space n_x > 0 | (n_x = 0, n_y > 0) | (n_x = n_y = 0, n_z > 0) of
// the sphere |n|^2 <= K^2; the other half contributes the same amount (S_-k is
// the conjugate of S_k), hence the factor 2 in G.  exp(i k.r) factorises into
// per-axis powers exp(i n_a theta_a), theta_a = 2 pi x_a / L.
//
// Work layout (MI355X-first, VALU-bound; no floating-point atomics):
//  * k_phase   builds per-particle tables of exp(i n theta_a), n = 0..KP-1, for the
//              three axes (x table pre-multiplied by q), in the caller's particle
//              order.  Powers come from FP64 recurrences: exp(i theta) inside blocks
//              of kQ, exp(i 2 kQ theta) from block to block, from FP64 sincos.
//  * k_sk      one block = one "unit" (64 rows x one segment of kQ values a = |n_z|)
//              times one particle chunk.  Lanes own rows; the particle loop is
//              wave-uniform, so exp(i a theta_z) for the segment is read through the
//              scalar path, while q exp(i n_x theta_x) exp(i n_y theta_y) per lane comes
//              from LDS tiles.  Each (particle, slot) costs four FMAs that serve both
//              +a and -a (the phases are conjugates).  Phases, products and sums
//              are FP64 in both precisions.
//  * k_sk_reduce sums the chunk partials in a fixed order, forms E_recip partials,
//              S_k (kept for inspection) and the per-slot gather coefficients.
//  * k_gather  lanes own particles; the loop over (segment, row) items is uniform so
//              the coefficients arrive through the scalar path; the 2 kQ vectors of an
//              item cost 8 FMAs per a (4 per k vector).
#include "ewald_internal.h"

namespace ewk {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr int kPhaseRows = 64;  // table rows (particle, axis) per phase block

template <typename R>
__device__ inline typename Cplx<R>::type make_c(double re, double im)
{
    typename Cplx<R>::type c;
    c.re = (R)re;
    c.im = (R)im;
    return c;
}

// ------------------------------------------------------------------ k_phase
// Two threads per table row (particle j, axis), each with two FP64 sincos
// (theta and kQ theta): thread h fills the blocks of kQ powers b = h, h + 2, ...
// The powers inside a block follow the FP64 recurrence from the block's anchor
// q exp(i kQ b theta); the anchors start at exp(i kQ h theta) and advance by
// exp(i 2 kQ theta) (at most kQ + KP / (2 kQ) + 1 rounding steps from an exact
// value).  The block's rows are staged in LDS and stored with consecutive
// threads on consecutive entries.
template <typename R>
__device__ __forceinline__ void phase_body(int bx, int by, int64_t n, double L, int KP, const double *__restrict__ pos,
                                           const double *__restrict__ qv, d4 *__restrict__ pr,
                                           typename Cplx<R>::type *__restrict__ tx,
                                           typename Cplx<R>::type *__restrict__ ty,
                                           typename Cplx<R>::type *__restrict__ tz)
{
    using C = typename Cplx<R>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    C *buf = reinterpret_cast<C *>(smem);  // [rows of the block][KP]
    const int rows = (int)blockDim.x / 2;
    const int lr = (int)threadIdx.x >> 1, h = (int)threadIdx.x & 1;
    // grid row = axis: a block's rows are consecutive particles of one table,
    // so its write-out is one contiguous run
    const int ax = (int)by;
    const int64_t r0 = (int64_t)bx * rows;
    const int64_t row = r0 + lr;
    if (row < n) {
        const int64_t j = row;
        const double qj = qv[j];
        const double x = wrap_coord(pos[3 * j + ax], L);
        if (ax == 0 && h == 0) {
            d4 r;
            r.a = x;
            r.b = wrap_coord(pos[3 * j + 1], L);
            r.c = wrap_coord(pos[3 * j + 2], L);
            r.d = qj;
            pr[j] = r;
        }
        const double th = (2.0 * kPi / L) * x;
        double s1, c1, s8, c8;
        sincos(th, &s1, &c1);
        sincos((double)kQ * th, &s8, &c8);
        const double scale = ax == 0 ? qj : 1.0;
        // anchor q exp(i kQ b theta) of block b = h; step exp(i 2 kQ theta)
        double ar = h ? scale * c8 : scale, ai = h ? scale * s8 : 0.0;
        const double c16 = c8 * c8 - s8 * s8, s16 = 2.0 * s8 * c8;
        C *dst = buf + (size_t)lr * KP;
        for (int b = kQ * h; b < KP; b += 2 * kQ) {
            double pr_ = ar, pi_ = ai;
#pragma unroll
            for (int k = 0; k < kQ; ++k) {
                dst[b + k] = make_c<R>(pr_, pi_);
                const double nr = pr_ * c1 - pi_ * s1;
                pi_ = pr_ * s1 + pi_ * c1;
                pr_ = nr;
            }
            const double na = ar * c16 - ai * s16;
            ai = ar * s16 + ai * c16;
            ar = na;
        }
    }
    __syncthreads();
    const int64_t nrows = n - r0 < rows ? n - r0 : rows;
    const int count = (int)nrows * KP;
    C *out = (ax == 0 ? tx : (ax == 1 ? ty : tz)) + r0 * KP;
    for (int e = (int)threadIdx.x; e < count; e += (int)blockDim.x) out[e] = buf[e];
}

template <typename R>
struct KPhase {
    static constexpr int kThreads = 2 * kPhaseRows;
    static constexpr int kWavesPerEu = 1;
    int64_t n;
    double L;
    int KP;
    const double *pos;
    const double *qv;
    d4 *pr;
    typename Cplx<R>::type *tx;
    typename Cplx<R>::type *ty;
    typename Cplx<R>::type *tz;
    __device__ void run(int bx, int by) const { phase_body<R>(bx, by, n, L, KP, pos, qv, pr, tx, ty, tz); }
    hipError_t one(hipStream_t s, dim3 grid, int threads, size_t smem) const;
};

template <typename R>
__global__ __launch_bounds__(2 * kPhaseRows) void k_phase(int64_t n, double L, int KP, const double *__restrict__ pos,
                                                          const double *__restrict__ qv, d4 *__restrict__ pr,
                                                          typename Cplx<R>::type *__restrict__ tx,
                                                          typename Cplx<R>::type *__restrict__ ty,
                                                          typename Cplx<R>::type *__restrict__ tz)
{
    phase_body<R>(blockIdx.x, blockIdx.y, n, L, KP, pos, qv, pr, tx, ty, tz);
}

template <typename R>
hipError_t KPhase<R>::one(hipStream_t s, dim3 grid, int threads, size_t smem) const
{
    hipLaunchKernelGGL((k_phase<R>), grid, dim3(threads), smem, s, n, L, KP, pos, qv, pr, tx, ty, tz);
    return hipGetLastError();
}

// --------------------------------------------------------------------- k_sk
// Block = kSkWaves waves on one unit (64 rows x one segment); the block's
// particle chunk is cut into tiles of `ts` particles and wave w takes tiles
// w, w + kSkWaves, ...  Each wave stages the x/y power tables of its own tile
// in a private, double-buffered LDS area (the next tile's global loads are in
// flight while the current tile is consumed), so no block barrier is needed
// until the final fixed-order reduction over the waves.  The z powers of the
// unit's segment are wave-uniform and come through the scalar path, prefetched
// one particle ahead; so are the lane's x/y entries.
constexpr int kSkStage = 4;  // staged table entries per lane and tile (upper bound)

// Operands of one particle for k_sk: the segment's kQ z powers (wave-uniform,
// scalar path) and the lane's x/y powers from the staged tile (LDS).
__device__ inline void load_ops(const c64 *__restrict__ zrow, const c64 *cur, int jj, int KP, int K1, int nx, int ay,
                                c64 (&z)[kQ], c64 &a, c64 &b)
{
#pragma unroll
    for (int k = 0; k < kQ; ++k) z[k] = zrow[(size_t)jj * KP + k];
    a = cur[jj * 2 * K1 + nx];
    b = cur[jj * 2 * K1 + ay];
}

// Scalar and LDS loads share one wait counter and scalar loads return out of
// order; this empty statement makes the prefetched operands due at this point
// (after the preceding FMAs) instead of letting the compiler sink the loads
// next to their use.  It contains no instructions.
__device__ inline void pin_ops(const c64 (&z)[kQ], const c64 &a, const c64 &b)
{
    asm volatile("" ::"s"(z[0].re), "s"(z[0].im), "s"(z[1].re), "s"(z[1].im), "s"(z[2].re), "s"(z[2].im),
                 "s"(z[3].re), "s"(z[3].im), "s"(z[4].re), "s"(z[4].im), "s"(z[5].re), "s"(z[5].im), "s"(z[6].re),
                 "s"(z[6].im), "s"(z[7].re), "s"(z[7].im), "v"(a.re), "v"(a.im), "v"(b.re), "v"(b.im));
}

// W = (q x-power)(y-power or its conjugate); accumulate the four real products
// that give both S(+a) and S(-a) for the kQ values of a in the segment.
__device__ inline void sk_fma(const c64 (&z)[kQ], const c64 &a, const c64 &b, double ysign, double (&A)[kQ],
                              double (&B)[kQ], double (&Cc)[kQ], double (&D)[kQ])
{
    const double bi = b.im * ysign;
    const double wr = a.re * b.re - a.im * bi;
    const double wi = a.re * bi + a.im * b.re;
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
        A[k] = fma(wr, z[k].re, A[k]);
        B[k] = fma(wi, z[k].im, B[k]);
        Cc[k] = fma(wr, z[k].im, Cc[k]);
        D[k] = fma(wi, z[k].re, D[k]);
    }
}


__device__ __forceinline__ void sk_body(int bx, int by, int64_t n, int chunk_len, int ts, int KP, int K1,
                                        const c64 *__restrict__ tx, const c64 *__restrict__ ty,
                                        const c64 *__restrict__ tz, const int *__restrict__ unit_group,
                                        const int *__restrict__ unit_seg, const int *__restrict__ row_nx,
                                        const int *__restrict__ row_ny, int n_rows, int n_units, int n_chunks,
                                        d4 *__restrict__ part)
{
    extern __shared__ __align__(32) unsigned char smem[];
    const int lane = threadIdx.x & (kLanes - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    const int per_tile = ts * 2 * K1;                                   // c64 entries in one tile
    c64 *buf = reinterpret_cast<c64 *>(smem) + (size_t)wave * 2 * per_tile;  // two buffers
    d4 *red = reinterpret_cast<d4 *>(smem);

    // logical block = chunk * n_units + unit, placed so that all units of a
    // chunk (which share its phase tables) run on one XCD
    const int lb = xcd_remap(bx, n_units * n_chunks);
    if (lb >= n_units * n_chunks) return;
    const int u = lb % n_units;
    const int chunk = lb / n_units;
    const int seg = unit_seg[u];
    const int r = unit_group[u] * kLanes + lane;
    int nx = 0, ny = 0;
    if (r < n_rows) {
        nx = row_nx[r];
        ny = row_ny[r];
    }
    const int ay = K1 + (ny < 0 ? -ny : ny);  // y entries follow the x entries of a particle
    const double ysign = ny < 0 ? -1.0 : 1.0;
    const int64_t j0 = (int64_t)chunk * chunk_len;
    const int64_t j1 = (j0 + chunk_len < n) ? j0 + chunk_len : n;
    const int n_tiles = j1 > j0 ? (int)((j1 - j0 + ts - 1) / ts) : 0;

    double A[kQ], B[kQ], Cc[kQ], D[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) A[k] = B[k] = Cc[k] = D[k] = 0.0;

    // Staging of one tile: entry e = lane + 64 k (k < kSkStage) is particle
    // e / (2 K1), table x or y, power e % K1; offsets are fixed per lane.
    static_assert(kSkStage == 4, "staging uses four named registers");
    int off[kSkStage];
    bool isy[kSkStage];
#pragma unroll
    for (int k = 0; k < kSkStage; ++k) {
        const int e = lane + k * kLanes;
        const int jj = e / (2 * K1), rem = e - jj * 2 * K1;
        isy[k] = rem >= K1;
        off[k] = jj * KP + (isy[k] ? rem - K1 : rem);
    }
    c64 st0, st1, st2, st3;
    auto ld = [&](int64_t tb, int cnt, int k) -> c64 {
        const int e = lane + k * kLanes;
        const int o = e < cnt ? off[k] : 0;  // clamp to the tile's first entry
        return (isy[k] && e < cnt ? ty : tx)[tb * KP + o];
    };
    auto fetch = [&](int t) {
        const int64_t tb = j0 + (int64_t)t * ts;
        const int cnt = (int)((j1 - tb) < ts ? (j1 - tb) : ts) * 2 * K1;
        st0 = ld(tb, cnt, 0);
        st1 = ld(tb, cnt, 1);
        st2 = ld(tb, cnt, 2);
        st3 = ld(tb, cnt, 3);
    };
    auto store = [&](int t, int slot) {
        const int64_t tb = j0 + (int64_t)t * ts;
        const int cnt = (int)((j1 - tb) < ts ? (j1 - tb) : ts) * 2 * K1;
        c64 *dst = buf + slot * per_tile;
        if (lane < cnt) dst[lane] = st0;
        if (lane + kLanes < cnt) dst[lane + kLanes] = st1;
        if (lane + 2 * kLanes < cnt) dst[lane + 2 * kLanes] = st2;
        if (lane + 3 * kLanes < cnt) dst[lane + 3 * kLanes] = st3;
    };

    int t = wave;
    if (t < n_tiles) {
        fetch(t);
        store(t, 0);
    }
    int slot = 0;
    for (; t < n_tiles; t += kSkWaves) {
        const int tn_next = t + kSkWaves;
        if (tn_next < n_tiles) fetch(tn_next);  // in flight during this tile
        __builtin_amdgcn_wave_barrier();
        const int64_t tb = j0 + (int64_t)t * ts;
        const int tn = (int)((j1 - tb) < ts ? (j1 - tb) : ts);
        const c64 *cur = buf + slot * per_tile;
        const c64 *zrow = tz + tb * KP + seg * kQ;
        // two alternating operand sets: the loads of one particle are issued
        // before the FMAs of the previous one and are made due after them
        c64 z0[kQ], z1[kQ], a0, b0, a1, b1;
        load_ops(zrow, cur, 0, KP, K1, nx, ay, z0, a0, b0);
        for (int jj = 0; jj < tn; jj += 2) {
            const int j1n = jj + 1 < tn ? jj + 1 : tn - 1;
            load_ops(zrow, cur, j1n, KP, K1, nx, ay, z1, a1, b1);
            sk_fma(z0, a0, b0, ysign, A, B, Cc, D);
            pin_ops(z1, a1, b1);
            const int j2n = jj + 2 < tn ? jj + 2 : tn - 1;
            load_ops(zrow, cur, j2n, KP, K1, nx, ay, z0, a0, b0);
            if (jj + 1 < tn) sk_fma(z1, a1, b1, ysign, A, B, Cc, D);
            pin_ops(z0, a0, b0);
        }
        if (tn_next < n_tiles) {
            slot ^= 1;
            __builtin_amdgcn_wave_barrier();
            store(tn_next, slot);
        }
    }
    // S(+a) = sum W z = (A - B, C + D);  S(-a) = sum W conj(z) = (A + B, D - C)
    d4 mine[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
        mine[k].a = A[k] - B[k];
        mine[k].b = Cc[k] + D[k];
        mine[k].c = A[k] + B[k];
        mine[k].d = D[k] - Cc[k];
    }
    // fixed-order sum over the block's waves through LDS (aliases the tiles)
    for (int w = 1; w < kSkWaves; ++w) {
        __syncthreads();
        if (wave == w) {
#pragma unroll
            for (int k = 0; k < kQ; ++k) red[k * kLanes + lane] = mine[k];
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int k = 0; k < kQ; ++k) {
                const d4 o = red[k * kLanes + lane];
                mine[k].a += o.a;
                mine[k].b += o.b;
                mine[k].c += o.c;
                mine[k].d += o.d;
            }
        }
    }
    if (wave == 0) {
        d4 *dst = part + ((size_t)chunk * n_units + u) * kQ * kLanes + lane;
#pragma unroll
        for (int k = 0; k < kQ; ++k) dst[k * kLanes] = mine[k];
    }
}

struct KSk {
    static constexpr int kThreads = kSkWaves *kLanes;
    static constexpr int kWavesPerEu = 1;
    int64_t n;
    int chunk_len;
    int ts;
    int KP;
    int K1;
    const c64 *tx;
    const c64 *ty;
    const c64 *tz;
    const int *unit_group;
    const int *unit_seg;
    const int *row_nx;
    const int *row_ny;
    int n_rows;
    int n_units;
    int n_chunks;
    d4 *part;
    __device__ void run(int bx, int by) const
    {
        sk_body(bx, by, n, chunk_len, ts, KP, K1, tx, ty, tz, unit_group, unit_seg, row_nx, row_ny, n_rows, n_units,
                n_chunks, part);
    }
    hipError_t one(hipStream_t s, dim3 grid, int threads, size_t smem) const;
};

__global__ __launch_bounds__(kSkWaves *kLanes) void k_sk(int64_t n, int chunk_len, int ts, int KP, int K1,
                                                         const c64 *__restrict__ tx, const c64 *__restrict__ ty,
                                                         const c64 *__restrict__ tz, const int *__restrict__ unit_group,
                                                         const int *__restrict__ unit_seg,
                                                         const int *__restrict__ row_nx, const int *__restrict__ row_ny,
                                                         int n_rows, int n_units, int n_chunks, d4 *__restrict__ part)
{
    sk_body(blockIdx.x, blockIdx.y, n, chunk_len, ts, KP, K1, tx, ty, tz, unit_group, unit_seg, row_nx, row_ny, n_rows,
            n_units, n_chunks, part);
}

hipError_t KSk::one(hipStream_t s, dim3 grid, int threads, size_t smem) const
{
    hipLaunchKernelGGL((k_sk), grid, dim3(threads), smem, s, n, chunk_len, ts, KP, K1, tx, ty, tz, unit_group, unit_seg,
                       row_nx, row_ny, n_rows, n_units, n_chunks, part);
    return hipGetLastError();
}

// ------------------------------------------------------------- k_sk_reduce
constexpr int kRedLanes = kRedSlotLanes;  // lanes cooperating on one slot

template <typename R>
__device__ __forceinline__ void sk_reduce_body(int bx, int by, int n_chunks, int n_units, int n_rows,
                                               const d4 *__restrict__ part, const int *__restrict__ unit_group,
                                               const int *__restrict__ unit_seg, const int *__restrict__ row_nx,
                                               const int *__restrict__ row_ny, const int *__restrict__ row_m,
                                               const int *__restrict__ row_item, const double *__restrict__ ck,
                                               d4 *__restrict__ sk, R *__restrict__ rec, R *__restrict__ mcoef,
                                               const int *__restrict__ row_mbase, double *__restrict__ erec_part)
{
    __shared__ double s_e[256];
    const int n_slots = n_units * kQ * kLanes;
    // kRedLanes lanes per slot: lane group c sums chunks c, c + kRedLanes, ...;
    // the partial sums are then combined by a fixed xor-shuffle tree.  A wave
    // takes kLanes / kRedLanes consecutive slots, so every load instruction
    // reads kRedLanes contiguous runs of slots.
    constexpr int kWaveSlots = kLanes / kRedLanes;
    const int ln = (int)threadIdx.x % kLanes;
    const int sub = ln / kWaveSlots;
    const int slot = bx * (256 / kRedLanes) + ((int)threadIdx.x / kLanes) * kWaveSlots + ln % kWaveSlots;
    const int cslot = slot < n_slots ? slot : n_slots - 1;
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int c = sub; c < n_chunks; c += kRedLanes) {
        const d4 p = part[(size_t)c * n_slots + cslot];
        s0 += p.a;
        s1 += p.b;
        s2 += p.c;
        s3 += p.d;
    }
#pragma unroll
    for (int w = kWaveSlots; w < kLanes; w <<= 1) {
        s0 += __shfl_xor(s0, w);
        s1 += __shfl_xor(s1, w);
        s2 += __shfl_xor(s2, w);
        s3 += __shfl_xor(s3, w);
    }
    double e = 0.0;
    if (slot < n_slots && sub == 0) {
        const int lane = slot & (kLanes - 1);
        const int uq = slot / kLanes;
        const int k = uq % kQ;
        const int u = uq / kQ;
        const int seg = unit_seg[u];
        const int r = unit_group[u] * kLanes + lane;
        const int a = seg * kQ + k;
        int nx = 0, ny = 0, m = -1;
        if (r < n_rows) {
            nx = row_nx[r];
            ny = row_ny[r];
            m = row_m[r];
        }
        const bool valid = a <= m;
        const bool axis = (nx == 0 && ny == 0);
        const bool vp = valid && !(axis && a == 0);  // (nx, ny, +a) in K+
        const bool vm = valid && a > 0 && !axis;     // (nx, ny, -a) in K+
        const double C = (vp || vm) ? ck[nx * nx + ny * ny + a * a] : 0.0;
        const double spr = vp ? s0 : 0.0, spi = vp ? s1 : 0.0;
        const double smr = vm ? s2 : 0.0, smi = vm ? s3 : 0.0;
        e = C * (spr * spr + spi * spi + smr * smr + smi * smi);
        d4 out;
        out.a = spr;
        out.b = spi;
        out.c = smr;
        out.d = smi;
        sk[slot] = out;
        if (r < n_rows && m >= seg * kQ) {
            // gather coefficients from a = conj(G+), b = conj(G-), G = 2 C S
            const double ar = 2.0 * C * spr, ai = -2.0 * C * spi;
            const double br = 2.0 * C * smr, bi = -2.0 * C * smi;
            const double cu = ar + br, cv = bi - ai, cs = ar - br, ct = ai + bi;
            const double w = (double)a;
            if (rec) {
                const int item = row_item[seg * n_rows + r];
                R *o = rec + ((size_t)item * kQ + k) * 8;
                o[0] = (R)cu;
                o[1] = (R)cv;
                o[2] = (R)cs;
                o[3] = (R)ct;
                o[4] = (R)(w * cs);
                o[5] = (R)(-w * ct);
                o[6] = (R)(w * cu);
                o[7] = (R)(-w * cv);
            }
            if (mcoef && a <= m) {
                // T_re = cu Re z + cv Im z, T_im = ct Re z + cs Im z,
                // Tz_re = a (cs Re z - ct Im z), Tz_im = a (cu Im z - cv Re z)
                R *o = mcoef + (size_t)row_mbase[r] + (size_t)(a >> 1) * kMBlock + (size_t)(a & 1) * 32;
                o[0] = (R)cu;
                o[16] = (R)cv;
                o[64] = (R)ct;
                o[64 + 16] = (R)cs;
                o[128] = (R)(w * cs);
                o[128 + 16] = (R)(-w * ct);
                o[192] = (R)(-w * cv);
                o[192 + 16] = (R)(w * cu);
            }
        }
    }
    s_e[threadIdx.x] = e;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s_e[threadIdx.x] += s_e[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) erec_part[bx] = s_e[0];
}

template <typename R>
struct KSkReduce {
    static constexpr int kThreads = 256;
    static constexpr int kWavesPerEu = 1;
    int n_chunks;
    int n_units;
    int n_rows;
    const d4 *part;
    const int *unit_group;
    const int *unit_seg;
    const int *row_nx;
    const int *row_ny;
    const int *row_m;
    const int *row_item;
    const double *ck;
    d4 *sk;
    R *rec;
    R *mcoef;
    const int *row_mbase;
    double *erec_part;
    __device__ void run(int bx, int by) const
    {
        sk_reduce_body<R>(bx, by, n_chunks, n_units, n_rows, part, unit_group, unit_seg, row_nx, row_ny, row_m,
                          row_item, ck, sk, rec, mcoef, row_mbase, erec_part);
    }
    hipError_t one(hipStream_t s, dim3 grid, int threads, size_t smem) const;
};

template <typename R>
__global__ __launch_bounds__(256) void k_sk_reduce(int n_chunks, int n_units, int n_rows, const d4 *__restrict__ part,
                                                   const int *__restrict__ unit_group, const int *__restrict__ unit_seg,
                                                   const int *__restrict__ row_nx, const int *__restrict__ row_ny,
                                                   const int *__restrict__ row_m, const int *__restrict__ row_item,
                                                   const double *__restrict__ ck, d4 *__restrict__ sk,
                                                   R *__restrict__ rec, R *__restrict__ mcoef,
                                                   const int *__restrict__ row_mbase, double *__restrict__ erec_part)
{
    sk_reduce_body<R>(blockIdx.x, blockIdx.y, n_chunks, n_units, n_rows, part, unit_group, unit_seg, row_nx, row_ny,
                      row_m, row_item, ck, sk, rec, mcoef, row_mbase, erec_part);
}

template <typename R>
hipError_t KSkReduce<R>::one(hipStream_t s, dim3 grid, int threads, size_t smem) const
{
    hipLaunchKernelGGL((k_sk_reduce<R>), grid, dim3(threads), smem, s, n_chunks, n_units, n_rows, part, unit_group,
                       unit_seg, row_nx, row_ny, row_m, row_item, ck, sk, rec, mcoef, row_mbase, erec_part);
    return hipGetLastError();
}

// ----------------------------------------------------------------- k_gather
// Lanes own particles; the loop over (segment, row) items is wave-uniform.  An
// item's coefficients (kQ values of a, 8 each) are consumed in four quarters of
// two a values; quarters alternate between two scalar register sets so that the
// loads of one quarter are in flight during the FMAs of the previous one.  The
// next item's packed (segment, n_x, n_y) word travels with its first quarter.
template <typename R>
__device__ inline void load_quarter(const R *__restrict__ rec, int g, R (&v)[16])
{
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = rec[(size_t)g * 16 + k];
}

template <typename R>
__device__ inline void pin_quarter(const R (&v)[16], int meta)
{
    asm volatile("" ::"s"(v[0]), "s"(v[1]), "s"(v[2]), "s"(v[3]), "s"(v[4]), "s"(v[5]), "s"(v[6]), "s"(v[7]),
                 "s"(v[8]), "s"(v[9]), "s"(v[10]), "s"(v[11]), "s"(v[12]), "s"(v[13]), "s"(v[14]), "s"(v[15]),
                 "s"(meta));
}

// T += sum over the quarter's two a values of the 8 coefficient products.
template <typename R>
__device__ inline void gather_fma(const R (&v)[16], const typename Cplx<R>::type *p, R &Tr, R &Ti, R &Zr, R &Zi)
{
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const R pr = p[h].re, pi = p[h].im;
        const R *c = v + 8 * h;
        Tr = fma(c[0], pr, Tr);
        Tr = fma(c[1], pi, Tr);
        Ti = fma(c[2], pi, Ti);
        Ti = fma(c[3], pr, Ti);
        Zr = fma(c[4], pr, Zr);
        Zr = fma(c[5], pi, Zr);
        Zi = fma(c[6], pi, Zi);
        Zi = fma(c[7], pr, Zi);
    }
}

template <typename R>
__device__ __forceinline__ void gather_body(int bx, int by, int64_t n, double L, int KP, const SplitTable &split,
                                            const d4 *__restrict__ pq, const c64 *__restrict__ tz,
                                            const int *__restrict__ item_meta, const R *__restrict__ rec,
                                            d4 *__restrict__ gpart)
{
    using C = typename Cplx<R>::type;
    const int64_t j = (int64_t)bx * 256 + threadIdx.x;
    const int sp = by;
    const int i0 = split.lo[sp], i1 = split.lo[sp + 1];
    const int64_t jj = j < n ? j : n - 1;
    const d4 r = pq[jj];
    const double gk = 2.0 * kPi / L;
    const double thx = gk * r.a, thy = gk * r.b;
    double sy, cy;
    sincos(thy, &sy, &cy);
    double ph = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    C p[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) p[k] = make_c<R>(0.0, 0.0);
    int cur_seg = -1, pnx = -1000000, pny = 0;
    double wr64 = 1.0, wi64 = 0.0;
    R qa[16], qb[16];
    int meta = 0;
    if (i0 < i1) {
        load_quarter(rec, 4 * i0, qa);
        meta = item_meta[i0];
    }
    for (int it = i0; it < i1; ++it) {
        const int s = meta >> 16, nx = (meta >> 8) & 0xff, ny = (meta & 0xff) - 128;
        if (s != cur_seg) {
            const c64 *src = tz + jj * KP + s * kQ;
#pragma unroll
            for (int k = 0; k < kQ; ++k) p[k] = make_c<R>(src[k].re, src[k].im);
            cur_seg = s;
            pnx = -1000000;
        }
        if (nx == pnx && ny == pny + 1) {
            const double t = wr64 * cy - wi64 * sy;
            wi64 = wr64 * sy + wi64 * cy;
            wr64 = t;
        } else {
            sincos((double)nx * thx + (double)ny * thy, &wi64, &wr64);
        }
        pnx = nx;
        pny = ny;
        R Tr = 0, Ti = 0, Zr = 0, Zi = 0;
        const int g = 4 * it;
        load_quarter(rec, g + 1, qb);
        gather_fma(qa, p + 0, Tr, Ti, Zr, Zi);
        pin_quarter(qb, 0);
        load_quarter(rec, g + 2, qa);
        gather_fma(qb, p + 2, Tr, Ti, Zr, Zi);
        pin_quarter(qa, 0);
        load_quarter(rec, g + 3, qb);
        gather_fma(qa, p + 4, Tr, Ti, Zr, Zi);
        pin_quarter(qb, 0);
        const int itn = it + 1 < i1 ? it + 1 : it;  // next item (clamped)
        load_quarter(rec, 4 * itn, qa);
        const int meta_n = item_meta[itn];
        gather_fma(qb, p + 6, Tr, Ti, Zr, Zi);
        pin_quarter(qa, meta_n);
        meta = meta_n;
        const R wr = (R)wr64, wi = (R)wi64;
        const R re = wr * Tr - wi * Ti;   // Re(w T)
        const R im = wr * Ti + wi * Tr;   // Im(w T)
        const R imz = wr * Zi + wi * Zr;  // Im(w Tz)
        ph += (double)re;
        fx += (double)nx * (double)im;
        fy += (double)ny * (double)im;
        fz += (double)imz;
    }
    if (j < n) {
        d4 o;
        o.a = ph;
        o.b = fx;
        o.c = fy;
        o.d = fz;
        gpart[(size_t)sp * n + j] = o;
    }
}

template <typename R>
struct KGather {
    static constexpr int kThreads = 256;
    static constexpr int kWavesPerEu = 1;
    int64_t n;
    double L;
    int KP;
    SplitTable split;
    const d4 *pq;
    const c64 *tz;
    const int *item_meta;
    const R *rec;
    d4 *gpart;
    __device__ void run(int bx, int by) const
    {
        gather_body<R>(bx, by, n, L, KP, split, pq, tz, item_meta, rec, gpart);
    }
    hipError_t one(hipStream_t s, dim3 grid, int threads, size_t smem) const;
};

template <typename R>
__global__ __launch_bounds__(256) void k_gather(int64_t n, double L, int KP, SplitTable split,
                                                const d4 *__restrict__ pq, const c64 *__restrict__ tz,
                                                const int *__restrict__ item_meta, const R *__restrict__ rec,
                                                d4 *__restrict__ gpart)
{
    gather_body<R>(blockIdx.x, blockIdx.y, n, L, KP, split, pq, tz, item_meta, rec, gpart);
}

template <typename R>
hipError_t KGather<R>::one(hipStream_t s, dim3 grid, int threads, size_t smem) const
{
    hipLaunchKernelGGL((k_gather<R>), grid, dim3(threads), smem, s, n, L, KP, split, pq, tz, item_meta, rec, gpart);
    return hipGetLastError();
}

}  // namespace

template <typename R>
int phase_rows(int KP)
{
    // rows per block: kPhaseRows, fewer when their LDS stage would pass 64 KB
    int rows = kPhaseRows;
    while (rows > 1 && (size_t)rows * KP * sizeof(typename Cplx<R>::type) > 64 * 1024) rows /= 2;
    return rows;
}

template <typename R>
hipError_t launch_phase(hipStream_t s, const RecipArgs &a, const double *pos, const double *q, d4 *pr,
                        typename Cplx<R>::type *tx, typename Cplx<R>::type *ty, typename Cplx<R>::type *tz)
{
    const int rows = phase_rows<R>(a.KP);
    return launch(s, dim3(ceil_div(a.n, rows), 3), 2 * rows, (size_t)rows * a.KP * sizeof(typename Cplx<R>::type),
                  KPhase<R>{a.n, a.L, a.KP, pos, q, pr, tx, ty, tz});
}

// LDS bytes of one structure-factor block: two staged tiles per wave, or the
// 16 KB cross-wave reduction buffer, whichever is larger.
size_t sk_smem_bytes(int ts, int K1)
{
    const size_t tab = (size_t)kSkWaves * 2 * ts * 2 * K1 * sizeof(c64);
    const size_t red = (size_t)kQ * kLanes * sizeof(d4);
    return tab > red ? tab : red;
}

// Particles per staged tile: the largest ts <= 8 whose 2*ts*K1 entries fit the
// per-lane staging registers (kSkStage per lane).
int sk_tile(int K1)
{
    int ts = kSkStage * kLanes / (2 * K1);
    if (ts > 8) ts = 8;
    return ts < 1 ? 1 : ts;
}

hipError_t launch_sk(hipStream_t s, const RecipArgs &a, int n_chunks, int chunk_len, const c64 *tx, const c64 *ty,
                     const c64 *tz, const int *unit_group, const int *unit_seg, const int *row_nx, const int *row_ny,
                     d4 *part)
{
    const int K1 = a.K + 1;
    const int ts = sk_tile(K1);
    return launch(s, dim3(xcd_grid(a.n_units * n_chunks)), kSkWaves * kLanes, sk_smem_bytes(ts, K1),
                  KSk{a.n, chunk_len, ts, a.KP, K1, tx, ty, tz, unit_group, unit_seg, row_nx, row_ny, a.n_rows,
                      a.n_units, n_chunks, part});
}

template <typename R>
hipError_t launch_sk_reduce(hipStream_t s, const RecipArgs &a, int n_chunks, const d4 *part, const int *unit_group,
                            const int *unit_seg, const int *row_nx, const int *row_ny, const int *row_m,
                            const int *row_item, const double *ck, d4 *sk, R *rec, R *mcoef, const int *row_mbase,
                            double *erec_part)
{
    return launch(s, dim3(ceil_div(a.n_slots, 256 / kRedLanes)), 256, 0,
                  KSkReduce<R>{n_chunks, a.n_units, a.n_rows, part, unit_group, unit_seg, row_nx, row_ny, row_m,
                               row_item, ck, sk, rec, mcoef, row_mbase, erec_part});
}

template <typename R>
hipError_t launch_gather(hipStream_t s, const RecipArgs &a, int n_split, const SplitTable &split, const d4 *pq,
                         const c64 *tz, const int *item_meta, const R *rec, d4 *gpart)
{
    return launch(s, dim3(ceil_div(a.n, 256), n_split), 256, 0,
                  KGather<R>{a.n, a.L, a.KP, split, pq, tz, item_meta, rec, gpart});
}

#define EWK_INSTANTIATE(R)                                                                                         \
    template int phase_rows<R>(int);                                                                               \
    template hipError_t launch_phase<R>(hipStream_t, const RecipArgs &, const double *, const double *, d4 *,     \
                                        Cplx<R>::type *, Cplx<R>::type *, Cplx<R>::type *);                        \
    template hipError_t launch_sk_reduce<R>(hipStream_t, const RecipArgs &, int, const d4 *, const int *,          \
                                            const int *, const int *, const int *, const int *, const int *,      \
                                            const double *, d4 *, R *, R *, const int *, double *);               \
    template hipError_t launch_gather<R>(hipStream_t, const RecipArgs &, int, const SplitTable &, const d4 *,      \
                                         const c64 *, const int *, const R *, d4 *);

EWK_INSTANTIATE(float)
EWK_INSTANTIATE(double)

}  // namespace ewk
