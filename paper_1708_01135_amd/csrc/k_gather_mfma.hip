// Reciprocal-space force gather on the matrix cores (section 3.1.2, Algorithm 2,
// with the per-axis factorisation of Eq. perf_mod1).
//
// For particle i and a half-space row (n_x, n_y) the gather needs
//   T_i  = sum_{n_z} z_i^{n_z} conj(G(n_x, n_y, n_z)),    z_i = exp(i 2 pi z_i / L),
//   Tz_i = sum_{n_z} n_z z_i^{n_z} conj(G(n_x, n_y, n_z)),
// and then, with P = exp(i (n_x theta_x + n_y theta_y)),
//   phi_i += Re(P T),  (F_x, F_y) += (n_x, n_y) Im(P T),  F_z += Im(P Tz).
// Pairing +-n_z (z^-a = conj z^a) folds each row's sums to a = 0..m with real
// coefficients on (Re z^a, Im z^a); over all rows and particles that is a real
// matrix product  [4 quantities x rows] x [2 (m+1)] . [2 (m+1)] x [particles],
// evaluated here with 16x16x4 MFMAs: rows on M (16 = 4 quads of 4 consecutive
// n_y at one n_x), particles on N (16 per sub-tile), and two a values per
// instruction on K.  Coefficients stream from L2, 256 contiguous values per
// (tile, a pair); the z powers of the block's particles are staged once in
// LDS.  Lane l owns particle l % 16 of each sub-tile and, in output register
// r, row 4 (l / 16) + r (FP32) or 4 r + l / 16 (FP64); the plan places quad
// l / 16's n_y offset r there.  The phase P of the quad's first row comes from
// one reduced FP64 argument and FP32 polynomials (FP32, 32-particle blocks),
// or from x^n and y^n tables (0 <= n <= k_max) that the block builds in LDS
// for its particles (FP64 recurrences from one sincos per eight powers; FP64,
// and FP32 64-particle blocks): one complex product instead of a sincos per
// quad and particle.  The other three
// rows follow by a recurrence along n_y.  Sums over rows are FP64 per lane,
// then reduced over the four lane groups and the block's waves in a fixed
// order.
//
// FP32 (MIXED): FP32 operands and MFMA accumulation over a, FP32 phases P,
// FP64 sums over rows.  FP64: every step in double (FP64 MFMA).
#include "ewald_internal.h"

namespace ewk {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr int kGmWaves = 4;

template <typename R>
struct Mfma;
template <>
struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ inline v4 mma(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
template <>
struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ inline v4 mma(double a, double b, v4 c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// e^{i theta} rounded to R.  FP64: the library sincos.  FP32: theta is reduced
// modulo pi/2 in FP64 (Cody-Waite, pi/2 split in two doubles whose first part
// has 33 significant bits, so k pi/2_hi is exact for |k| < 2^20), the remainder
// (|r| <= pi/4) is rounded to FP32 and sin, cos are their Taylor series to r^9 and
// r^10 (truncation below 1e-9 on [-pi/4, pi/4]); the quadrant k mod 4 permutes
// and signs the pair.  Error about 1 FP32 ulp of the result, as for the rounding
// of an FP64 value.
template <typename R>
__device__ inline void row_phase(double th, R &c, R &s);
template <>
__device__ inline void row_phase<double>(double th, double &c, double &s)
{
    sincos(th, &s, &c);
}
template <>
__device__ inline void row_phase<float>(double th, float &c, float &s)
{
    constexpr double kTwoOverPi = 0.63661977236758134308;
    constexpr double kPio2Hi = 1.5707963267341256141662597656e+00;  // 33-bit head of pi/2
    constexpr double kPio2Lo = 6.0771005065061922358e-11;           // pi/2 - kPio2Hi
    const double k = rint(th * kTwoOverPi);
    const float r = (float)(fma(-k, kPio2Lo, fma(-k, kPio2Hi, th)));
    const float r2 = r * r;
    // sin r = r (1 - r^2/3! + r^4/5! - r^6/7! + r^8/9!), cos r = 1 - r^2/2! + ... + r^8/8! - r^10/10!
    const float sp = fmaf(fmaf(fmaf(fmaf(2.7557319e-6f, r2, -1.9841270e-4f), r2, 8.3333333e-3f), r2, -1.6666667e-1f), r2, 1.0f);
    const float cp = fmaf(fmaf(fmaf(fmaf(fmaf(-2.7557319e-7f, r2, 2.4801587e-5f), r2, -1.3888889e-3f), r2, 4.1666667e-2f), r2, -0.5f), r2, 1.0f);
    const float sr = r * sp;
    const int q = (int)k & 3;
    const float a = (q & 1) ? cp : sr;   // sin of theta up to sign
    const float b = (q & 1) ? sr : cp;   // cos of theta up to sign
    s = (q & 2) ? -a : a;
    c = (q == 1 || q == 2) ? -b : b;
}

template <typename R>
struct RC {
    R re, im;
};

// Where the phases come from: LDS tables for the FP64 gather (a library FP64
// sincos per quad and particle cost more than building them) and for FP32
// blocks of 64 particles (large systems: a block then meets every tile, so the
// tables' setup is spread over many epilogues; 64^3 took 1464 against 1521 us
// per gather, rel_F 3.25e-7 either way); row_phase for FP32 blocks of 32
// (tables made rock salt 32^3 slower).
template <typename R, int NP>
constexpr bool gather_tables()
{
    return sizeof(R) == 8 || NP == 64;
}

// padded LDS stride of one k component for blocks of NP particles: the four
// 16-lane groups of a read start 16 (FP32) or 32 (FP64) banks apart
constexpr int zs_stride(int np) { return np + 16; }

template <typename R, int NP>
__device__ __forceinline__ void gather_mfma_body(int bx, int by, int64_t n, double L, int KP, int K, int nap_max,
                                                 const SplitTable &split, const d4 *__restrict__ pq,
                                                 const c64 *__restrict__ tz, const MTile *__restrict__ tiles,
                                                 const R *__restrict__ coef, d4 *__restrict__ gpart)
{
    using V = typename Mfma<R>::v4;
    constexpr int NSUB = NP / 16;
    constexpr int ZS = zs_stride(NP);
    extern __shared__ __align__(16) unsigned char smem[];
    R *zs = reinterpret_cast<R *>(smem);  // [nap_max][4][ZS]

    const int lane = (int)threadIdx.x & (kLanes - 1);
    // wave index made visibly uniform: tile loads and loop control stay scalar
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kLanes);
    const int64_t p0 = (int64_t)bx * NP;

    // z powers of the block's particles: entry (p, k, col) = Re/Im z^(2p + k/2),
    // loaded eight per thread at a time (indices clamped in bounds, stores
    // predicated) so that the loads are in flight together
    constexpr int kBatch = 8;
    const int total = nap_max * 4 * NP;
    for (int e0 = (int)threadIdx.x; e0 < total; e0 += kBatch * kGmWaves * kLanes) {
        double zv[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            int e = e0 + u * kGmWaves * kLanes;
            e = e < total ? e : total - 1;
            const int col = e % NP, k = (e / NP) & 3, p = e / (4 * NP);
            int64_t j = p0 + col;
            j = j < n ? j : n - 1;
            zv[u] = reinterpret_cast<const double *>(tz + j * KP + 2 * p + (k >> 1))[k & 1];
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int e = e0 + u * kGmWaves * kLanes;
            if (e < total) {
                const int col = e % NP, k = (e / NP) & 3, p = e / (4 * NP);
                zs[(p * 4 + k) * ZS + col] = (R)zv[u];
            }
        }
    }

    const double gk = 2.0 * kPi / L;
    constexpr bool kTab = gather_tables<R, NP>();
    // FP64: x^n and y^n (n <= K) of the block's particles, entry (axis, n, col)
    // at ptab[(axis (K + 1) + n) NP + col].  Thread task (axis, block of eight
    // powers, col): one sincos at the block's first power and one for the
    // step, then the recurrence.
    const int K1 = K + 1;
    RC<R> *ptab = reinterpret_cast<RC<R> *>(zs + (size_t)nap_max * 4 * ZS);
    if constexpr (kTab) {
        const int nb8 = (K1 + 7) / 8;
        for (int idx = (int)threadIdx.x; idx < 2 * nb8 * NP; idx += kGmWaves * kLanes) {
            const int col = idx % NP, b = (idx / NP) % nb8, axis = idx / (NP * nb8);
            int64_t j = p0 + col;
            j = j < n ? j : n - 1;
            const d4 r = pq[j];
            const double th = gk * (axis ? r.b : r.a);
            double s0, c0, s1, c1;
            sincos((double)(8 * b) * th, &s0, &c0);
            sincos(th, &s1, &c1);
            RC<R> *o = ptab + ((size_t)axis * K1 + 8 * b) * NP + col;
            const int cnt = K1 - 8 * b < 8 ? K1 - 8 * b : 8;
            for (int m = 0; m < cnt; ++m) {
                o[(size_t)m * NP] = RC<R>{(R)c0, (R)s0};
                const double t = c0 * c1 - s0 * s1;
                s0 = c0 * s1 + s0 * c1;
                c0 = t;
            }
        }
    }
    double thx[NSUB], thy[NSUB];
    R cy[NSUB], sy[NSUB];
    double ph[NSUB], fx[NSUB], fy[NSUB], fz[NSUB];
#pragma unroll
    for (int s = 0; s < NSUB; ++s) {
        ph[s] = fx[s] = fy[s] = fz[s] = 0.0;
        if constexpr (!kTab) {
            int64_t j = p0 + 16 * s + (lane & 15);
            j = j < n ? j : n - 1;
            const d4 r = pq[j];
            thx[s] = gk * r.a;
            thy[s] = gk * r.b;
            double sn, cs;
            sincos(thy[s], &sn, &cs);
            cy[s] = (R)cs;
            sy[s] = (R)sn;
        }
    }
    __syncthreads();
    if constexpr (kTab) {
        // the n_y step of the row recurrence: y^1 of the lane's particles
#pragma unroll
        for (int s = 0; s < NSUB; ++s) {
            const RC<R> y1 = ptab[((size_t)K1 + (K1 > 1 ? 1 : 0)) * NP + 16 * s + (lane & 15)];
            cy[s] = y1.re;
            sy[s] = y1.im;
        }
    }

    const int g = lane >> 4;  // quad of this lane
    const int lo = split.lo[by], hi = split.lo[by + 1];
    const R *zl = zs + g * ZS + (lane & 15);
    for (int t = lo + w; t < hi; t += kGmWaves) {
        const MTile tl = tiles[t];
        V acc[4][NSUB];
        const R *cb = coef + (size_t)tl.base * kMBlock + lane;
        // operands two a pairs ahead, in three named register sets (the loop is
        // unrolled by three, so no set is copied and each load has a whole pair
        // of MFMAs, about 500 cycles, to arrive)
        auto load_pair = [&](int p, R (&c)[4], R (&z)[NSUB]) {
            const R *cp = cb + (size_t)p * kMBlock;
#pragma unroll
            for (int q = 0; q < 4; ++q) c[q] = cp[64 * q];
#pragma unroll
            for (int s = 0; s < NSUB; ++s) z[s] = zl[p * 4 * ZS + 16 * s];
        };
        auto mfma_pair = [&](const R (&c)[4], const R (&z)[NSUB]) {
#pragma unroll
            for (int s = 0; s < NSUB; ++s) {
                acc[0][s] = Mfma<R>::mma(c[0], z[s], acc[0][s]);
                acc[1][s] = Mfma<R>::mma(c[1], z[s], acc[1][s]);
                acc[2][s] = Mfma<R>::mma(c[2], z[s], acc[2][s]);
                acc[3][s] = Mfma<R>::mma(c[3], z[s], acc[3][s]);
            }
        };
        // the first a pair starts the accumulators (zero C operand)
        auto mfma_first = [&](const R (&c)[4], const R (&z)[NSUB]) {
#pragma unroll
            for (int s = 0; s < NSUB; ++s) {
                acc[0][s] = Mfma<R>::mma(c[0], z[s], V{0, 0, 0, 0});
                acc[1][s] = Mfma<R>::mma(c[1], z[s], V{0, 0, 0, 0});
                acc[2][s] = Mfma<R>::mma(c[2], z[s], V{0, 0, 0, 0});
                acc[3][s] = Mfma<R>::mma(c[3], z[s], V{0, 0, 0, 0});
            }
        };
        const int nap = tl.nap, last = nap - 1;  // nap >= 1
        R c0[4], z0[NSUB], c1[4], z1[NSUB], c2[4], z2[NSUB];
        load_pair(0, c0, z0);
        load_pair(last < 1 ? last : 1, c1, z1);
        load_pair(last < 2 ? last : 2, c2, z2);
        mfma_first(c0, z0);
        if (1 < nap) {
            load_pair(last < 3 ? last : 3, c0, z0);
            mfma_pair(c1, z1);
        }
        if (2 < nap) {
            load_pair(last < 4 ? last : 4, c1, z1);
            mfma_pair(c2, z2);
        }
        for (int p = 3; p < nap; p += 3) {
            load_pair(p + 2 < last ? p + 2 : last, c2, z2);
            mfma_pair(c0, z0);
            if (p + 1 < nap) {
                load_pair(p + 3 < last ? p + 3 : last, c0, z0);
                mfma_pair(c1, z1);
            }
            if (p + 2 < nap) {
                load_pair(p + 4 < last ? p + 4 : last, c1, z1);
                mfma_pair(c2, z2);
            }
        }
        // epilogue: rows n_y0 + r (r = 0..3) of this lane's quad; the four rows are
        // summed in R, then added to the FP64 accumulators
        const int qd = g == 0 ? tl.quad[0] : (g == 1 ? tl.quad[1] : (g == 2 ? tl.quad[2] : tl.quad[3]));
        const int nx = qd >> 16, ny0 = (qd & 0xffff) - 32768;
#pragma unroll
        for (int s = 0; s < NSUB; ++s) {
            R pr, pi;
            if constexpr (kTab) {  // P = x^nx y^ny0, y^-a = conj y^a
                const int ay = ny0 < 0 ? -ny0 : ny0;
                const RC<R> xv = ptab[(size_t)nx * NP + 16 * s + (lane & 15)];
                const RC<R> yv = ptab[((size_t)K1 + ay) * NP + 16 * s + (lane & 15)];
                const R yi = ny0 < 0 ? -yv.im : yv.im;
                pr = xv.re * yv.re - xv.im * yi;
                pi = xv.re * yi + xv.im * yv.re;
            } else {
                row_phase<R>((double)nx * thx[s] + (double)ny0 * thy[s], pr, pi);
            }
            R sre = 0, sim = 0, srim = 0, simz = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const R tr = acc[0][s][r], ti = acc[1][s][r], zr = acc[2][s][r], zi = acc[3][s][r];
                const R re = pr * tr - pi * ti;   // Re(P T)
                const R im = pr * ti + pi * tr;   // Im(P T)
                const R imz = pr * zi + pi * zr;  // Im(P Tz)
                sre += re;
                sim += im;
                srim += (R)r * im;
                simz += imz;
                if (r < 3) {
                    const R npr = pr * cy[s] - pi * sy[s];
                    pi = pr * sy[s] + pi * cy[s];
                    pr = npr;
                }
            }
            ph[s] += (double)sre;
            fx[s] += (double)nx * (double)sim;
            fy[s] += (double)ny0 * (double)sim + (double)srim;
            fz[s] += (double)simz;
        }
    }

    // fixed-order sums: the four lane groups, then the block's waves
#pragma unroll
    for (int s = 0; s < NSUB; ++s) {
#pragma unroll
        for (int m = 16; m < kLanes; m <<= 1) {
            ph[s] += __shfl_xor(ph[s], m);
            fx[s] += __shfl_xor(fx[s], m);
            fy[s] += __shfl_xor(fy[s], m);
            fz[s] += __shfl_xor(fz[s], m);
        }
    }
    __syncthreads();  // the z stage is reused for the cross-wave sums
    d4 *red = reinterpret_cast<d4 *>(smem);  // [kGmWaves][NP]
    if (lane < 16) {
#pragma unroll
        for (int s = 0; s < NSUB; ++s) {
            d4 v;
            v.a = ph[s];
            v.b = fx[s];
            v.c = fy[s];
            v.d = fz[s];
            red[w * NP + 16 * s + lane] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < NP) {
        const int col = (int)threadIdx.x;
        d4 o = red[col];
#pragma unroll
        for (int u = 1; u < kGmWaves; ++u) {
            const d4 v = red[u * NP + col];
            o.a += v.a;
            o.b += v.b;
            o.c += v.c;
            o.d += v.d;
        }
        const int64_t j = p0 + col;
        if (j < n) gpart[(size_t)by * n + j] = o;
    }
}

template <typename R, int NP>
struct KGatherMfma {
    static constexpr int kThreads = kGmWaves * kLanes;
    static constexpr int kWavesPerEu = 1;
    int64_t n;
    double L;
    int KP;
    int K;
    int nap_max;
    SplitTable split;
    const d4 *pq;
    const c64 *tz;
    const MTile *tiles;
    const R *coef;
    d4 *gpart;
    __device__ void run(int bx, int by) const
    {
        gather_mfma_body<R, NP>(bx, by, n, L, KP, K, nap_max, split, pq, tz, tiles, coef, gpart);
    }
    hipError_t one(hipStream_t s, dim3 grid, int threads, size_t smem) const;
};

template <typename R, int NP>
__global__ __launch_bounds__(kGmWaves * kLanes) void k_gather_mfma(int64_t n, double L, int KP, int K, int nap_max,
                                                                   SplitTable split, const d4 *__restrict__ pq,
                                                                   const c64 *__restrict__ tz,
                                                                   const MTile *__restrict__ tiles,
                                                                   const R *__restrict__ coef, d4 *__restrict__ gpart)
{
    gather_mfma_body<R, NP>(blockIdx.x, blockIdx.y, n, L, KP, K, nap_max, split, pq, tz, tiles, coef, gpart);
}

template <typename R, int NP>
hipError_t KGatherMfma<R, NP>::one(hipStream_t s, dim3 grid, int threads, size_t smem) const
{
    hipLaunchKernelGGL((k_gather_mfma<R, NP>), grid, dim3(threads), smem, s, n, L, KP, K, nap_max, split, pq, tz, tiles,
                       coef, gpart);
    return hipGetLastError();
}

}  // namespace

size_t gather_mfma_stage_bytes(int nap_max, int np, bool fp64)
{
    return (size_t)nap_max * 4 * zs_stride(np) * (fp64 ? sizeof(double) : sizeof(float));
}

size_t gather_mfma_smem_bytes(int nap_max, int np, int K, bool fp64)
{
    const bool tables = fp64 ? gather_tables<double, 32>() : (np == 64 ? gather_tables<float, 64>() : gather_tables<float, 32>());
    const size_t tab = tables ? (size_t)2 * (K + 1) * np * (fp64 ? sizeof(RC<double>) : sizeof(RC<float>)) : 0;
    const size_t stage = gather_mfma_stage_bytes(nap_max, np, fp64) + tab;
    const size_t red = (size_t)kGmWaves * np * sizeof(d4);
    return stage > red ? stage : red;
}

template <typename R>
hipError_t launch_gather_mfma(hipStream_t s, const RecipArgs &a, int n_split, const SplitTable &split, int nap_max,
                              const d4 *pq, const c64 *tz, const MTile *tiles, const R *mcoef, d4 *gpart)
{
    const bool fp64 = sizeof(R) == 8;
    const int np = gather_mfma_particles(a.n, fp64);
    const int blocks = ceil_div(a.n, np);
    const size_t smem = gather_mfma_smem_bytes(nap_max, np, a.K, fp64);
    if (np == 64)
        return launch(s, dim3(blocks, n_split), kGmWaves * kLanes, smem,
                      KGatherMfma<R, 64>{a.n, a.L, a.KP, a.K, nap_max, split, pq, tz, tiles, mcoef, gpart});
    return launch(s, dim3(blocks, n_split), kGmWaves * kLanes, smem,
                  KGatherMfma<R, 32>{a.n, a.L, a.KP, a.K, nap_max, split, pq, tz, tiles, mcoef, gpart});
}

template hipError_t launch_gather_mfma<float>(hipStream_t, const RecipArgs &, int, const SplitTable &, int,
                                              const d4 *, const c64 *, const MTile *, const float *, d4 *);
template hipError_t launch_gather_mfma<double>(hipStream_t, const RecipArgs &, int, const SplitTable &, int,
                                               const d4 *, const c64 *, const MTile *, const double *, d4 *);

}  // namespace ewk
