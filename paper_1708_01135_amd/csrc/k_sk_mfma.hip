// Structure factor on the matrix cores (section 3.1.2, Algorithm 1 and the
// per-axis factorisation of Eq. perf_mod1), FP64 throughout.
//
// For a half-space row (n_x, n_y) and a = |n_z|,
//   S(+a) = sum_j U_j z_j^a,  S(-a) = sum_j U_j conj(z_j^a),  U_j = q_j x_j^{n_x} y_j^{n_y},
// so with the four real sums P1 = sum Re U Re z, P2 = sum Im U Im z,
// P3 = sum Re U Im z, P4 = sum Im U Re z:
//   S(+a) = (P1 - P2, P3 + P4),  S(-a) = (P1 + P2, P4 - P3).
// Over particles that is a real matrix product [rows x (Re U, Im U)] .
// [(Re z^a, Im z^a) x a].  For k_max >= 24 it is evaluated with 16x16x4 FP64
// MFMAs: M = 8 rows x (Re U, Im U), N = 8 values of a x (Re z, Im z), K = 4
// particles; for k_max <= 23 with 4x4x4 FP64 MFMAs (the wide variant below).
//
// Rows are taken in the structure-factor order (sorted by m, 64 to a group);
// a wave owns a tile of 8 consecutive rows and accumulates every block of 8
// a values the tile needs; a block of kSmWaves waves covers kSmWaves tiles and
// one particle chunk.  The plan deals the tiles to (block, wave) so that the
// two waves sharing a SIMD (w and w + 4) pair a heavy tile with a light one
// and every block gets a similar mix: the waves of a block meet at a barrier
// after every staged sub-chunk, so a block runs at the pace of its busiest
// SIMD.  The block stages the q x^n, y^n and z^n tables
// of P particles at a time in LDS (sk_mfma_particles).  The partial sums of the chunk are
// written in the slot layout of the vector kernel (unit = (row group, a
// segment), a mod 8, row mod 64), so the same fixed-order reduction follows.
#include "ewald_internal.h"

namespace ewk {

namespace {

typedef double dv4 __attribute__((ext_vector_type(4)));

// One staged sub-chunk against the wave's tile: NAT blocks of 8 values of a,
// fixed at compile time so that the quad loop has no branches.
template <int NAT>
__device__ __forceinline__ void sk_tile_pass(const c64 *__restrict__ st, int per, int KP, int P, int nx, int ay,
                                             double ysg, bool a_im, int kq, int bofs, int bim, dv4 (&acc)[kSmNat])
{
    // two quads per step (P is a multiple of 8): both quads' operand reads are
    // issued before their MFMAs
    for (int pq = 0; pq < P; pq += 8) {
        double aop[2];
        const double *zrow[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int p = pq + 4 * h + kq;
            const c64 xv = st[p * KP + nx];
            const c64 yv = st[per + p * KP + ay];
            const double yi = ysg * yv.im;
            aop[h] = a_im ? xv.re * yi + xv.im * yv.re : xv.re * yv.re - xv.im * yi;
            zrow[h] = reinterpret_cast<const double *>(st + 2 * per + p * KP + bofs) + bim;
        }
        double z0[NAT], z1[NAT];
#pragma unroll
        for (int b = 0; b < NAT; ++b) {
            z0[b] = zrow[0][2 * kSmRows * b];
            z1[b] = zrow[1][2 * kSmRows * b];
        }
#pragma unroll
        for (int b = 0; b < NAT; ++b) acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop[0], z0[b], acc[b], 0, 0, 0);
#pragma unroll
        for (int b = 0; b < NAT; ++b) acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop[1], z1[b], acc[b], 0, 0, 0);
    }
}

__global__ __launch_bounds__(kSmWaves *kLanes, 4) void k_sk_mfma(int64_t n, int KP, int P, int n_rows, int n_groups,
                                                              int n_chunks, int chunk_len,
                                                              const c64 *__restrict__ tx, const c64 *__restrict__ ty,
                                                              const c64 *__restrict__ tz,
                                                              const int *__restrict__ row_nx,
                                                              const int *__restrict__ row_ny,
                                                              const int *__restrict__ row_m,
                                                              const int *__restrict__ unit_base,
                                                              const int *__restrict__ tile_of, int n_slots,
                                                              d4 *__restrict__ part)
{
    extern __shared__ __align__(16) unsigned char smem[];
    c64 *st = reinterpret_cast<c64 *>(smem);  // [3][P][KP]: q x^n, y^n, z^n
    const int nb = n_groups * n_chunks;
    // the row groups of one chunk read the same particle tables: give every XCD
    // a contiguous range of (chunk, group) pairs
    const int bid = xcd_remap(blockIdx.x, nb);
    if (bid >= nb) return;  // padding block (uniform over the block)
    const int chunk = bid / n_groups, grp = bid % n_groups;
    const int64_t j_lo = (int64_t)chunk * chunk_len;
    const int64_t j_hi = j_lo + chunk_len < n ? j_lo + chunk_len : n;

    const int lane = (int)threadIdx.x & (kLanes - 1);
    const int w = (int)threadIdx.x / kLanes;
    // first row of the wave's tile (tiles are dealt to waves by the plan so that
    // the block's SIMD pairs carry similar work; -1: no tile)
    const int tt = tile_of[grp * kSmWaves + w];
    const int tile_row0 = tt < 0 ? n_rows : tt * kSmRows;
    // A operand: row tile_row0 + (lane % 8), component lane / 8 % 2 of U
    const int ra = tile_row0 + (lane & 7);
    const bool ra_ok = ra < n_rows;
    const int nx = ra_ok ? row_nx[ra] : 0;
    const int nyv = ra_ok ? row_ny[ra] : 0;
    const int ay = nyv < 0 ? -nyv : nyv;
    const double ysg = nyv < 0 ? -1.0 : 1.0;
    const bool a_im = (lane >> 3) & 1;
    // B operand: a offset (lane % 16) / 2, component lane % 2 of z^a
    const int bofs = (lane & 15) >> 1, bim = lane & 1;
    const int kq = lane >> 4;  // particle of the quad (K index)
    const int nat = tile_row0 < n_rows ? (row_m[tile_row0] + kSmRows) / kSmRows : 0;  // blocks of 8 a values

    dv4 acc[kSmNat];
#pragma unroll
    for (int b = 0; b < kSmNat; ++b) acc[b] = dv4{0, 0, 0, 0};

    // Staging: the P particles' entries of each table are contiguous, so a
    // sub-chunk is three straight copies.  The next sub-chunk is loaded into
    // registers (at most kSmStage entries per thread) while the current one is
    // consumed from LDS; entries of particles past the chunk are zero (their U
    // vanishes).
    const int per = P * KP;
    constexpr int kStride = kSmWaves * kLanes;
    // this thread's staging entries: table and offset are the same for every
    // sub-chunk (only the first particle moves)
    const c64 *sbase[kSmStage];
    int soff[kSmStage];
    bool suse[kSmStage];
#pragma unroll
    for (int u = 0; u < kSmStage; ++u) {
        const int e = (int)threadIdx.x + u * kStride;
        const int tab = e < per ? 0 : (e < 2 * per ? 1 : 2);
        suse[u] = e < 3 * per;
        soff[u] = e - tab * per;
        sbase[u] = tab == 0 ? tx : (tab == 1 ? ty : tz);
    }
    c64 v[kSmStage];
    auto valid_of = [&](int64_t j0) { return (int)((j_hi - j0 < P ? j_hi - j0 : P) * KP); };
    // raw loads only: the zero fill is applied when the registers are stored, so
    // nothing waits for these loads before the next sub-chunk's store
    auto load_stage = [&](int64_t j0) {
        const int valid = valid_of(j0);
#pragma unroll
        for (int u = 0; u < kSmStage; ++u) {
            const bool ok = suse[u] && soff[u] < valid;
            v[u] = sbase[u][j0 * KP + (ok ? soff[u] : 0)];
        }
    };
    if (j_lo < j_hi) load_stage(j_lo);
    for (int64_t j0 = j_lo; j0 < j_hi; j0 += P) {
        __syncthreads();  // the previous sub-chunk is consumed
        const int valid = valid_of(j0);
#pragma unroll
        for (int u = 0; u < kSmStage; ++u) {
            if (suse[u]) {
                const bool ok = soff[u] < valid;
                c64 t;
                t.re = ok ? v[u].re : 0.0;
                t.im = ok ? v[u].im : 0.0;
                st[threadIdx.x + u * kStride] = t;
            }
        }
        __syncthreads();
        if (j0 + P < j_hi) load_stage(j0 + P);
        switch (nat) {  // wave-uniform
        case 1: sk_tile_pass<1>(st, per, KP, P, nx, ay, ysg, a_im, kq, bofs, bim, acc); break;
        case 2: sk_tile_pass<2>(st, per, KP, P, nx, ay, ysg, a_im, kq, bofs, bim, acc); break;
        case 3: sk_tile_pass<3>(st, per, KP, P, nx, ay, ysg, a_im, kq, bofs, bim, acc); break;
        case 4: sk_tile_pass<4>(st, per, KP, P, nx, ay, ysg, a_im, kq, bofs, bim, acc); break;
        case 5: sk_tile_pass<5>(st, per, KP, P, nx, ay, ysg, a_im, kq, bofs, bim, acc); break;
        case 6: sk_tile_pass<6>(st, per, KP, P, nx, ay, ysg, a_im, kq, bofs, bim, acc); break;
        default: break;
        }
    }

    // Output register r of lane l holds row (l / 16) + 4 r of the 16 M entries:
    // r = 0, 1 -> Re U of tile rows g, g + 4; r = 2, 3 -> Im U of the same rows
    // (g = l / 16), against column (a offset, component) = ((l % 16) / 2, l % 2).
    // The partner lane l ^ 1 holds the other z component.
    const int g = lane >> 4;
#pragma unroll
    for (int b = 0; b < kSmNat; ++b) {
        if (b >= nat) break;
        const double pu0 = __shfl_xor(acc[b][2], 1), pu1 = __shfl_xor(acc[b][3], 1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int r = tile_row0 + g + 4 * h;
            const double ur = acc[b][h], ui = h ? pu1 : pu0;
            // Re z column: S+re = P1 - P2, S-re = P1 + P2;  Im z column: S+im = P3 + P4, S-im = P4 - P3
            const double v1 = bim ? ur + ui : ur - ui;
            const double v2 = bim ? ui - ur : ur + ui;
            if (r < n_rows) {
                const int unit = unit_base[r / kLanes] + b;
                const int slot = (unit * kQ + bofs) * kLanes + (r & (kLanes - 1));
                double *o = reinterpret_cast<double *>(part + (size_t)chunk * n_slots + slot);
                o[bim] = v1;
                o[2 + bim] = v2;
            }
        }
    }
}

// Wide-tile variant for k_max <= 23, on the FP64 4x4x4 instruction (four
// independent 4x4x4 products per instruction, block g = (l / 4) % 4): a wave owns
// 16 rows and takes the values of a two at a time.  Lane l supplies A = U of row
// l % 16 (block (l / 4) % 4, A row l % 4) for particle l / 16 of the quad (the
// K index), and B = component l % 2 of z^(2b + (l % 4) / 2) of the same particle
// (every block gets the same B); two instructions per quad and pair b, one with
// Re U and one with Im U.  The output of lane l is row 4 ((l / 4) % 4) + l / 16
// of the tile against column l % 4.  Pairs of a waste at most one column of a
// row (the 8-wide blocks of the 16x16x4 form wasted 22 % of the (row, a) pairs
// at k_max = 20), and on this part the 4x4x4 instruction sustains about 1.45x
// the FP64 rate of the 16x16x4 one.
template <int NAP>
__device__ __forceinline__ void sk_wide_pass(const c64 *__restrict__ st, int per, int KP, int P, int nx, int ay,
                                             double ysg, int kq, int zc, double (&are)[kSmNapWide],
                                             double (&aim)[kSmNapWide])
{
    for (int pq = 0; pq < P; pq += 4) {
        const int p = pq + kq;
        const c64 xv = st[p * KP + nx];
        const c64 yv = st[per + p * KP + ay];
        const double yi = ysg * yv.im;
        const double ur = xv.re * yv.re - xv.im * yi;
        const double ui = xv.re * yi + xv.im * yv.re;
        const double *zrow = reinterpret_cast<const double *>(st + 2 * per + p * KP) + zc;
        double z[NAP];
#pragma unroll
        for (int b = 0; b < NAP; ++b) z[b] = zrow[4 * b];
#pragma unroll
        for (int b = 0; b < NAP; ++b) {
            are[b] = __builtin_amdgcn_mfma_f64_4x4x4f64(ur, z[b], are[b], 0, 0, 0);
            aim[b] = __builtin_amdgcn_mfma_f64_4x4x4f64(ui, z[b], aim[b], 0, 0, 0);
        }
    }
}

__global__ __launch_bounds__(kSmWaves *kLanes, 2) void k_sk_mfma_wide(int64_t n, int KP, int P, int n_rows,
                                                                     int n_rblocks, int n_chunks, int chunk_len,
                                                                     const c64 *__restrict__ tx,
                                                                     const c64 *__restrict__ ty,
                                                                     const c64 *__restrict__ tz,
                                                                     const int *__restrict__ row_nx,
                                                                     const int *__restrict__ row_ny,
                                                                     const int *__restrict__ row_m,
                                                                     const int *__restrict__ unit_base,
                                                                     const int *__restrict__ tile_of, int n_slots,
                                                                     d4 *__restrict__ part)
{
    extern __shared__ __align__(16) unsigned char smem[];
    c64 *st = reinterpret_cast<c64 *>(smem);  // [3][P][KP]: q x^n, y^n, z^n
    const int nb = n_rblocks * n_chunks;
    const int bid = xcd_remap(blockIdx.x, nb);
    if (bid >= nb) return;  // padding block (uniform over the block)
    const int chunk = bid / n_rblocks, rblk = bid % n_rblocks;
    const int64_t j_lo = (int64_t)chunk * chunk_len;
    const int64_t j_hi = j_lo + chunk_len < n ? j_lo + chunk_len : n;

    const int lane = (int)threadIdx.x & (kLanes - 1);
    const int w = (int)threadIdx.x / kLanes;
    const int tt = tile_of[rblk * kSmWaves + w];  // the wave's 16-row tile (-1: none)
    const int tile_row0 = tt < 0 ? n_rows : tt * 16;
    // A operand: row tile_row0 + lane % 16 (both parts of its U)
    const int ra = tile_row0 + (lane & 15);
    const bool ra_ok = ra < n_rows;
    const int nx = ra_ok ? row_nx[ra] : 0;
    const int nyv = ra_ok ? row_ny[ra] : 0;
    const int ay = nyv < 0 ? -nyv : nyv;
    const double ysg = nyv < 0 ? -1.0 : 1.0;
    const int zc = lane & 3;  // B column: z^(2b + zc / 2), component zc % 2
    const int kq = lane >> 4;
    const int nap = tile_row0 < n_rows ? (row_m[tile_row0] + 2) / 2 : 0;  // pairs of a values

    double are[kSmNapWide], aim[kSmNapWide];
#pragma unroll
    for (int b = 0; b < kSmNapWide; ++b) are[b] = aim[b] = 0.0;

    // Staging as in the 8-row kernel, kSmStageWide entries per thread.
    const int per = P * KP;
    constexpr int kStride = kSmWaves * kLanes;
    const c64 *sbase[kSmStageWide];
    int soff[kSmStageWide];
    bool suse[kSmStageWide];
#pragma unroll
    for (int u = 0; u < kSmStageWide; ++u) {
        const int e = (int)threadIdx.x + u * kStride;
        const int tab = e < per ? 0 : (e < 2 * per ? 1 : 2);
        suse[u] = e < 3 * per;
        soff[u] = e - tab * per;
        sbase[u] = tab == 0 ? tx : (tab == 1 ? ty : tz);
    }
    c64 v[kSmStageWide];
    auto valid_of = [&](int64_t j0) { return (int)((j_hi - j0 < P ? j_hi - j0 : P) * KP); };
    auto load_stage = [&](int64_t j0) {
        const int valid = valid_of(j0);
#pragma unroll
        for (int u = 0; u < kSmStageWide; ++u) {
            const bool ok = suse[u] && soff[u] < valid;
            v[u] = sbase[u][j0 * KP + (ok ? soff[u] : 0)];
        }
    };
    if (j_lo < j_hi) load_stage(j_lo);
    for (int64_t j0 = j_lo; j0 < j_hi; j0 += P) {
        __syncthreads();
        const int valid = valid_of(j0);
#pragma unroll
        for (int u = 0; u < kSmStageWide; ++u) {
            if (suse[u]) {
                const bool ok = soff[u] < valid;
                c64 t;
                t.re = ok ? v[u].re : 0.0;
                t.im = ok ? v[u].im : 0.0;
                st[threadIdx.x + u * kStride] = t;
            }
        }
        __syncthreads();
        if (j0 + P < j_hi) load_stage(j0 + P);
        switch (nap) {  // wave-uniform
        case 1: sk_wide_pass<1>(st, per, KP, P, nx, ay, ysg, kq, zc, are, aim); break;
        case 2: sk_wide_pass<2>(st, per, KP, P, nx, ay, ysg, kq, zc, are, aim); break;
        case 3: sk_wide_pass<3>(st, per, KP, P, nx, ay, ysg, kq, zc, are, aim); break;
        case 4: sk_wide_pass<4>(st, per, KP, P, nx, ay, ysg, kq, zc, are, aim); break;
        case 5: sk_wide_pass<5>(st, per, KP, P, nx, ay, ysg, kq, zc, are, aim); break;
        case 6: sk_wide_pass<6>(st, per, KP, P, nx, ay, ysg, kq, zc, are, aim); break;
        case 7: sk_wide_pass<7>(st, per, KP, P, nx, ay, ysg, kq, zc, are, aim); break;
        case 8: sk_wide_pass<8>(st, per, KP, P, nx, ay, ysg, kq, zc, are, aim); break;
        case 9: sk_wide_pass<9>(st, per, KP, P, nx, ay, ysg, kq, zc, are, aim); break;
        case 10: sk_wide_pass<10>(st, per, KP, P, nx, ay, ysg, kq, zc, are, aim); break;
        case 11: sk_wide_pass<11>(st, per, KP, P, nx, ay, ysg, kq, zc, are, aim); break;
        case 12: sk_wide_pass<12>(st, per, KP, P, nx, ay, ysg, kq, zc, are, aim); break;
        default: break;
        }
    }

    // lane l: row 4 ((l / 4) % 4) + l / 16 of the tile, a = 2b + (l % 4) / 2,
    // component l % 2; the partner lane l ^ 1 holds the other z component
    const int r = tile_row0 + 4 * ((lane >> 2) & 3) + (lane >> 4);
    const int aoff = (lane >> 1) & 1, bim = lane & 1;
#pragma unroll
    for (int b = 0; b < kSmNapWide; ++b) {
        const double ur = are[b];
        const double ui = __shfl_xor(aim[b], 1);  // partner's Im U with the other z part
        // Re z column: S+re = P1 - P2, S-re = P1 + P2;  Im z column: S+im = P3 + P4, S-im = P4 - P3
        const double v1 = bim ? ur + ui : ur - ui;
        const double v2 = bim ? ui - ur : ur + ui;
        const int a = 2 * b + aoff;
        if (b < nap && r < n_rows) {
            const int unit = unit_base[r / kLanes] + (a >> 3);
            const int slot = (unit * kQ + (a & 7)) * kLanes + (r & (kLanes - 1));
            double *o = reinterpret_cast<double *>(part + (size_t)chunk * n_slots + slot);
            o[bim] = v1;
            o[2 + bim] = v2;
        }
    }
}

}  // namespace

// Particles per staged sub-chunk: the largest of 64, 48 (16-row kernel only),
// 32, 16, 8 whose three tables (3 P KP entries) fit the kernel's staged entries
// per thread; a multiple of 8 (two quads per step).  0 if even 8 do not fit.
int sk_mfma_particles(int KP)
{
    const bool wide = KP <= kSmRows * kSmNatWide;
    const int cap = (wide ? kSmStageWide : kSmStage) * kSmWaves * kLanes;
    static const int kCand[5] = {64, 48, 32, 16, 8};
    for (int c = wide ? 0 : 2; c < 5; ++c)
        if (3 * kCand[c] * KP <= cap) return kCand[c];
    return 0;
}

size_t sk_mfma_smem_bytes(int KP) { return (size_t)3 * sk_mfma_particles(KP) * KP * sizeof(c64); }

hipError_t launch_sk_mfma(hipStream_t s, const RecipArgs &a, int n_groups, int n_chunks, int chunk_len,
                          const c64 *tx, const c64 *ty, const c64 *tz, const int *row_nx, const int *row_ny,
                          const int *row_m, const int *unit_base, const int *tile_of, d4 *part)
{
    const int P = sk_mfma_particles(a.KP);
    if (a.KP <= kSmRows * kSmNatWide) {
        const int n_rblocks = (a.n_rows + 2 * kLanes - 1) / (2 * kLanes);
        hipLaunchKernelGGL(k_sk_mfma_wide, dim3(xcd_grid(n_rblocks * n_chunks)), dim3(kSmWaves * kLanes),
                           sk_mfma_smem_bytes(a.KP), s, a.n, a.KP, P, a.n_rows, n_rblocks, n_chunks, chunk_len, tx, ty,
                           tz, row_nx, row_ny, row_m, unit_base, tile_of, a.n_slots, part);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_sk_mfma, dim3(xcd_grid(n_groups * n_chunks)), dim3(kSmWaves * kLanes), sk_mfma_smem_bytes(a.KP),
                       s, a.n, a.KP, P, a.n_rows, n_groups, n_chunks, chunk_len, tx, ty, tz, row_nx, row_ny, row_m,
                       unit_base, tile_of, a.n_slots, part);
    return hipGetLastError();
}

}  // namespace ewk
