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
//              three axes (x table pre-multiplied by q).  Powers come from an FP64
//              recurrence re-anchored every kQ steps at exp(i kQ m theta) taken from
//              FP64 sincos, then rounded to the table type.
//  * k_sk      one block = one "unit" (64 rows x one segment of kQ values a = |n_z|)
//              times one particle chunk.  Lanes own rows; the particle loop is
//              wave-uniform, so exp(i a theta_z) for the segment is read through the
//              scalar path, while q exp(i n_x theta_x) exp(i n_y theta_y) per lane comes
//              from LDS tiles.  Each (particle, slot) costs four FMAs that serve both
//              +a and -a (the phases are conjugates).  FP32 partials over at most
//              tile/kSkWaves particles are folded into FP64 (mixed precision).
//  * k_sk_reduce sums the chunk partials in a fixed order, forms E_recip partials,
//              S_k (kept for inspection) and the per-slot gather coefficients.
//  * k_gather  lanes own particles; the loop over (segment, row) items is uniform so
//              the coefficients arrive through the scalar path; the 2 kQ vectors of an
//              item cost 8 FMAs per a (4 per k vector).
#include "ewald_internal.h"

namespace ewk {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

template <typename R>
__device__ inline typename Cplx<R>::type make_c(double re, double im)
{
    typename Cplx<R>::type c;
    c.re = (R)re;
    c.im = (R)im;
    return c;
}

// ------------------------------------------------------------------ k_phase
template <typename R>
__global__ __launch_bounds__(256) void k_phase(int64_t n, double L, int KP, const d4 *__restrict__ pq,
                                               typename Cplx<R>::type *__restrict__ tx,
                                               typename Cplx<R>::type *__restrict__ ty,
                                               typename Cplx<R>::type *__restrict__ tz)
{
    const int nb = KP / kQ;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n * 3 * nb) return;
    const int b = (int)(t % nb);
    const int64_t ja = t / nb;
    const int ax = (int)(ja % 3);
    const int64_t j = ja / 3;
    const d4 r = pq[j];
    const double x = ax == 0 ? r.a : (ax == 1 ? r.b : r.c);
    const double th = (2.0 * kPi / L) * x;
    double s0, c0, sa, ca;
    sincos(th, &s0, &c0);
    sincos((double)(kQ * b) * th, &sa, &ca);
    const double scale = ax == 0 ? r.d : 1.0;
    typename Cplx<R>::type *out = (ax == 0 ? tx : (ax == 1 ? ty : tz)) + j * KP + kQ * b;
    double pr = ca, pi = sa;
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
        out[k] = make_c<R>(scale * pr, scale * pi);
        const double nr = pr * c0 - pi * s0;
        pi = pr * s0 + pi * c0;
        pr = nr;
    }
}

// --------------------------------------------------------------------- k_sk
template <typename R>
__global__ __launch_bounds__(kSkWaves *kLanes) void k_sk(int64_t n, int chunk_len, int tile, int KP, int K1,
                                                         const typename Cplx<R>::type *__restrict__ tx,
                                                         const typename Cplx<R>::type *__restrict__ ty,
                                                         const typename Cplx<R>::type *__restrict__ tz,
                                                         const int *__restrict__ unit_group,
                                                         const int *__restrict__ unit_seg,
                                                         const int *__restrict__ row_nx,
                                                         const int *__restrict__ row_ny, int n_rows, int n_units,
                                                         d4 *__restrict__ part)
{
    using C = typename Cplx<R>::type;
    extern __shared__ __align__(32) unsigned char smem[];
    C *lx = reinterpret_cast<C *>(smem);
    C *ly = lx + (size_t)tile * K1;
    d4 *red = reinterpret_cast<d4 *>(smem);

    const int lane = threadIdx.x & (kLanes - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    const int u = blockIdx.x;
    const int g = unit_group[u];
    const int seg = unit_seg[u];
    const int r = g * kLanes + lane;
    int nx = 0, ny = 0;
    if (r < n_rows) {
        nx = row_nx[r];
        ny = row_ny[r];
    }
    const int ay = ny < 0 ? -ny : ny;
    const R ysign = ny < 0 ? R(-1) : R(1);
    const int64_t j0 = (int64_t)blockIdx.y * chunk_len;
    const int64_t j1 = (j0 + chunk_len < n) ? j0 + chunk_len : n;

    R A[kQ], B[kQ], Cc[kQ], D[kQ];
    double Pr[kQ], Pi[kQ], Mr[kQ], Mi[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
        A[k] = B[k] = Cc[k] = D[k] = R(0);
        Pr[k] = Pi[k] = Mr[k] = Mi[k] = 0.0;
    }

    for (int64_t t0 = j0; t0 < j1; t0 += tile) {
        const int tn = (int)((j1 - t0) < tile ? (j1 - t0) : tile);
        __syncthreads();
        for (int e = threadIdx.x; e < tn * K1; e += kSkWaves * kLanes) {
            const int jj = e / K1;
            const int m = e - jj * K1;
            lx[e] = tx[(t0 + jj) * KP + m];
            ly[e] = ty[(t0 + jj) * KP + m];
        }
        __syncthreads();
        for (int jj = wave; jj < tn; jj += kSkWaves) {
            const C a = lx[jj * K1 + nx];
            const C b = ly[jj * K1 + ay];
            const R bi = b.im * ysign;
            const R wr = a.re * b.re - a.im * bi;
            const R wi = a.re * bi + a.im * b.re;
            const C *zp = tz + (t0 + jj) * KP + seg * kQ;  // wave-uniform address
#pragma unroll
            for (int k = 0; k < kQ; ++k) {
                const C z = zp[k];
                A[k] = fma(wr, z.re, A[k]);
                B[k] = fma(wi, z.im, B[k]);
                Cc[k] = fma(wr, z.im, Cc[k]);
                D[k] = fma(wi, z.re, D[k]);
            }
        }
        if constexpr (sizeof(R) == 4) {
            // fold the FP32 partial (<= tile / kSkWaves particles) into FP64
#pragma unroll
            for (int k = 0; k < kQ; ++k) {
                Pr[k] += (double)A[k] - (double)B[k];
                Pi[k] += (double)Cc[k] + (double)D[k];
                Mr[k] += (double)A[k] + (double)B[k];
                Mi[k] += (double)D[k] - (double)Cc[k];
                A[k] = B[k] = Cc[k] = D[k] = R(0);
            }
        }
    }
    d4 mine[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
        if constexpr (sizeof(R) == 4) {
            mine[k].a = Pr[k];
            mine[k].b = Pi[k];
            mine[k].c = Mr[k];
            mine[k].d = Mi[k];
        } else {
            // S(+a) = sum W z = (A - B, C + D);  S(-a) = sum W conj(z) = (A + B, D - C)
            mine[k].a = (double)A[k] - (double)B[k];
            mine[k].b = (double)Cc[k] + (double)D[k];
            mine[k].c = (double)A[k] + (double)B[k];
            mine[k].d = (double)D[k] - (double)Cc[k];
        }
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
        d4 *dst = part + ((size_t)blockIdx.y * n_units + u) * kQ * kLanes + lane;
#pragma unroll
        for (int k = 0; k < kQ; ++k) dst[k * kLanes] = mine[k];
    }
}

// ------------------------------------------------------------- k_sk_reduce
template <typename R>
__global__ __launch_bounds__(256) void k_sk_reduce(int n_chunks, int n_units, int n_rows, const d4 *__restrict__ part,
                                                   const int *__restrict__ unit_group,
                                                   const int *__restrict__ unit_seg, const int *__restrict__ row_nx,
                                                   const int *__restrict__ row_ny, const int *__restrict__ row_m,
                                                   const int *__restrict__ row_item, const double *__restrict__ ck,
                                                   d4 *__restrict__ sk, R *__restrict__ rec,
                                                   double *__restrict__ erec_part)
{
    __shared__ double s_e[256];
    const int n_slots = n_units * kQ * kLanes;
    const int slot = blockIdx.x * 256 + threadIdx.x;
    double e = 0.0;
    if (slot < n_slots) {
        const int lane = slot & (kLanes - 1);
        const int uq = slot / kLanes;
        const int k = uq % kQ;
        const int u = uq / kQ;
        double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        for (int c = 0; c < n_chunks; ++c) {
            const d4 p = part[(size_t)c * n_slots + slot];
            s0 += p.a;
            s1 += p.b;
            s2 += p.c;
            s3 += p.d;
        }
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
            const int item = row_item[seg * n_rows + r];
            // gather coefficients from a = conj(G+), b = conj(G-), G = 2 C S
            const double ar = 2.0 * C * spr, ai = -2.0 * C * spi;
            const double br = 2.0 * C * smr, bi = -2.0 * C * smi;
            const double cu = ar + br, cv = bi - ai, cs = ar - br, ct = ai + bi;
            const double w = (double)a;
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
    }
    s_e[threadIdx.x] = e;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s_e[threadIdx.x] += s_e[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) erec_part[blockIdx.x] = s_e[0];
}

// ----------------------------------------------------------------- k_gather
template <typename R>
__global__ __launch_bounds__(256) void k_gather(int64_t n, double L, int KP, SplitTable split,
                                                const d4 *__restrict__ pq,
                                                const typename Cplx<R>::type *__restrict__ tz,
                                                const int *__restrict__ item_nx, const int *__restrict__ item_ny,
                                                const int *__restrict__ item_seg, const R *__restrict__ rec,
                                                d4 *__restrict__ gpart)
{
    using C = typename Cplx<R>::type;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int sp = blockIdx.y;
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
    for (int it = i0; it < i1; ++it) {
        const int nx = item_nx[it], ny = item_ny[it], s = item_seg[it];
        if (s != cur_seg) {
            const C *src = tz + jj * KP + s * kQ;
#pragma unroll
            for (int k = 0; k < kQ; ++k) p[k] = src[k];
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
        const R wr = (R)wr64, wi = (R)wi64;
        const R *rr = rec + (size_t)it * kQ * 8;  // wave-uniform
        R Tr = 0, Ti = 0, Zr = 0, Zi = 0;
#pragma unroll
        for (int k = 0; k < kQ; ++k) {
            const R pr = p[k].re, pi = p[k].im;
            Tr = fma(rr[8 * k + 0], pr, Tr);
            Tr = fma(rr[8 * k + 1], pi, Tr);
            Ti = fma(rr[8 * k + 2], pi, Ti);
            Ti = fma(rr[8 * k + 3], pr, Ti);
            Zr = fma(rr[8 * k + 4], pr, Zr);
            Zr = fma(rr[8 * k + 5], pi, Zr);
            Zi = fma(rr[8 * k + 6], pi, Zi);
            Zi = fma(rr[8 * k + 7], pr, Zi);
        }
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

}  // namespace

template <typename R>
hipError_t launch_phase(hipStream_t s, const RecipArgs &a, const d4 *pq, typename Cplx<R>::type *tx,
                        typename Cplx<R>::type *ty, typename Cplx<R>::type *tz)
{
    const int64_t total = a.n * 3 * (a.KP / kQ);
    hipLaunchKernelGGL(k_phase<R>, dim3(ceil_div(total, 256)), dim3(256), 0, s, a.n, a.L, a.KP, pq, tx, ty, tz);
    return hipGetLastError();
}

template <typename R>
size_t sk_smem_bytes(int tile, int K1)
{
    const size_t tab = 2 * (size_t)tile * K1 * sizeof(typename Cplx<R>::type);
    const size_t red = (size_t)kQ * kLanes * sizeof(d4);
    return tab > red ? tab : red;
}

template <typename R>
hipError_t launch_sk(hipStream_t s, const RecipArgs &a, int n_chunks, int chunk_len, int tile,
                     const typename Cplx<R>::type *tx, const typename Cplx<R>::type *ty,
                     const typename Cplx<R>::type *tz, const int *unit_group, const int *unit_seg,
                     const int *row_nx, const int *row_ny, d4 *part)
{
    const int K1 = a.K + 1;
    hipLaunchKernelGGL(k_sk<R>, dim3(a.n_units, n_chunks), dim3(kSkWaves * kLanes), sk_smem_bytes<R>(tile, K1), s,
                       a.n, chunk_len, tile, a.KP, K1, tx, ty, tz, unit_group, unit_seg, row_nx, row_ny, a.n_rows,
                       a.n_units, part);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_sk_reduce(hipStream_t s, const RecipArgs &a, int n_chunks, const d4 *part, const int *unit_group,
                            const int *unit_seg, const int *row_nx, const int *row_ny, const int *row_m,
                            const int *row_item, const double *ck, d4 *sk, R *rec, double *erec_part)
{
    hipLaunchKernelGGL(k_sk_reduce<R>, dim3(ceil_div(a.n_slots, 256)), dim3(256), 0, s, n_chunks, a.n_units,
                       a.n_rows, part, unit_group, unit_seg, row_nx, row_ny, row_m, row_item, ck, sk, rec,
                       erec_part);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_gather(hipStream_t s, const RecipArgs &a, int n_split, const SplitTable &split, const d4 *pq,
                         const typename Cplx<R>::type *tz, const int *item_nx, const int *item_ny,
                         const int *item_seg, const R *rec, d4 *gpart)
{
    hipLaunchKernelGGL(k_gather<R>, dim3(ceil_div(a.n, 256), n_split), dim3(256), 0, s, a.n, a.L, a.KP, split, pq,
                       tz, item_nx, item_ny, item_seg, rec, gpart);
    return hipGetLastError();
}

#define EWK_INSTANTIATE(R)                                                                                         \
    template hipError_t launch_phase<R>(hipStream_t, const RecipArgs &, const d4 *, Cplx<R>::type *,             \
                                        Cplx<R>::type *, Cplx<R>::type *);                                         \
    template size_t sk_smem_bytes<R>(int, int);                                                                    \
    template hipError_t launch_sk<R>(hipStream_t, const RecipArgs &, int, int, int, const Cplx<R>::type *,         \
                                     const Cplx<R>::type *, const Cplx<R>::type *, const int *, const int *,      \
                                     const int *, const int *, d4 *);                                              \
    template hipError_t launch_sk_reduce<R>(hipStream_t, const RecipArgs &, int, const d4 *, const int *,          \
                                            const int *, const int *, const int *, const int *, const int *,      \
                                            const double *, d4 *, R *, double *);                                  \
    template hipError_t launch_gather<R>(hipStream_t, const RecipArgs &, int, const SplitTable &, const d4 *,      \
                                         const Cplx<R>::type *, const int *, const int *, const int *, const R *, \
                                         d4 *);

EWK_INSTANTIATE(float)
EWK_INSTANTIATE(double)

}  // namespace ewk
