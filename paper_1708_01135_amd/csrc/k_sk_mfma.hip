// Structure factor on the matrix cores (section 3.1.2, Algorithm 1 and the
// per-axis factorisation of Eq. perf_mod1), FP64 throughout.
//
// For a half-space row (n_x, n_y) and a = |n_z|,
//   S(+a) = sum_j U_j z_j^a,  S(-a) = sum_j U_j conj(z_j^a),  U_j = q_j x_j^{n_x} y_j^{n_y},
// so with the four real sums P1 = sum Re U Re z, P2 = sum Im U Im z,
// P3 = sum Re U Im z, P4 = sum Im U Re z:
//   S(+a) = (P1 - P2, P3 + P4),  S(-a) = (P1 + P2, P4 - P3).
// Over particles that is a real matrix product [rows x (Re U, Im U)] .
// [(Re z^a, Im z^a) x a], evaluated with FP64 4x4x4 MFMAs (k_max <= 47).
//
// Rows are taken in the structure-factor order (sorted by m); a wave owns a
// tile of 16 consecutive rows and accumulates every pair of a values the tile
// needs; a block of kSmWaves waves covers 128 rows and one particle chunk.  The
// plan deals the tiles to (block, wave) so that the two waves sharing a SIMD (w
// and w + 4) pair a heavy tile with a light one and every block gets a similar
// mix: the waves of a block meet at a barrier after every staged sub-chunk, so
// a block runs at the pace of its busiest SIMD.  The block stages the q x^n,
// y^n and z^n tables of P particles at a time in LDS (sk_mfma_particles).  The
// partial sums of the chunk are written in the slot layout of the vector
// kernel (unit = (64-row group, a segment), a mod 8, row mod 64), so the same
// fixed-order reduction follows.
#include "ewald_internal.h"

namespace ewk {

namespace {

// One staged sub-chunk against the wave's tile, on the FP64 4x4x4 instruction
// (four independent 4x4x4 products per instruction, block g = (l / 4) % 4): a
// wave owns 16 rows and takes the values of a two at a time.  Lane l supplies
// A = U of row l % 16 (block (l / 4) % 4, A row l % 4) for particle l / 16 of
// the quad (the K index), and B = component l % 2 of z^(2b + (l % 4) / 2) of the
// same particle (every block gets the same B); two instructions per quad and
// pair b, one with Re U and one with Im U.  The output of lane l is row 4 ((l / 4) % 4) + l / 16
// of the tile against column l % 4.  Pairs of a waste at most one column of a
// row (the 8-wide blocks of the 16x16x4 form wasted 22 % of the (row, a) pairs
// at k_max = 20), and on this part the 4x4x4 instruction sustains about 1.45x
// the FP64 rate of the 16x16x4 one.
template <int NAP, int NMAX>
__device__ __forceinline__ void sk_tile_pass(const c64 *__restrict__ st, int per, int KP, int P, int nx, int ay,
                                             double ysg, int kq, int zc, double (&are)[NMAX], double (&aim)[NMAX])
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

// The pass for the tile's pairs of a (wave-uniform), fixed at compile time so
// that the quad loop has no branches.
template <int NMAX, int NAP = 1>
__device__ __forceinline__ void sk_tile_dispatch(int nap, const c64 *__restrict__ st, int per, int KP, int P, int nx,
                                                 int ay, double ysg, int kq, int zc, double (&are)[NMAX],
                                                 double (&aim)[NMAX])
{
    if constexpr (NAP <= NMAX) {
        if (nap == NAP)
            sk_tile_pass<NAP, NMAX>(st, per, KP, P, nx, ay, ysg, kq, zc, are, aim);
        else
            sk_tile_dispatch<NMAX, NAP + 1>(nap, st, per, KP, P, nx, ay, ysg, kq, zc, are, aim);
    }
}

// NMAX: the most pairs of a per row the instance holds (kSmNapSmall for
// k_max < 2 kSmNapSmall, kSmNap otherwise): fewer accumulators leave more of
// the SIMD's registers to the real-space kernels that run beside it.
template <int NMAX>
__global__ __launch_bounds__(kSmWaves *kLanes, 2) void k_sk_mfma(int64_t n, int KP, int P, int n_rows, int n_rblocks,
                                                              int n_chunks, int chunk_len, const c64 *__restrict__ tx,
                                                              const c64 *__restrict__ ty, const c64 *__restrict__ tz,
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
    const int tile_row0 = tt < 0 ? n_rows : tt * kSmTileRows;
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

    double are[NMAX], aim[NMAX];
#pragma unroll
    for (int b = 0; b < NMAX; ++b) are[b] = aim[b] = 0.0;

    // Staging: the three tables of a sub-chunk are each P KP contiguous
    // entries; thread t stages entries t, t + 512, ... of each (at most
    // kSmStage / 3).  A whole sub-chunk (all but a chunk's last) needs no
    // clamping or zero fill.  Entry slots past P KP read entry 0 and are not
    // stored.
    constexpr int kStride = kSmWaves * kLanes;
    constexpr int kPer = kSmStage / 3;
    const int per = P * KP;
    const c64 *tab[3] = {tx, ty, tz};
    int eidx[kPer];
    bool euse[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int e = (int)threadIdx.x + k * kStride;
        euse[k] = e < per;
        eidx[k] = euse[k] ? e : 0;
    }
    c64 v[3][kPer];
    auto valid_of = [&](int64_t j0) { return (int)((j_hi - j0 < P ? j_hi - j0 : P) * KP); };
    auto load_stage = [&](int64_t j0) {
        const int valid = valid_of(j0);
        const int64_t o = j0 * KP;
        if (valid == per) {  // wave-uniform
#pragma unroll
            for (int t = 0; t < 3; ++t)
#pragma unroll
                for (int k = 0; k < kPer; ++k) v[t][k] = tab[t][o + eidx[k]];
        } else {
#pragma unroll
            for (int t = 0; t < 3; ++t)
#pragma unroll
                for (int k = 0; k < kPer; ++k) v[t][k] = tab[t][o + (eidx[k] < valid ? eidx[k] : 0)];
        }
    };
    if (j_lo < j_hi) load_stage(j_lo);
    for (int64_t j0 = j_lo; j0 < j_hi; j0 += P) {
        __syncthreads();
        const int valid = valid_of(j0);
        if (valid == per) {  // wave-uniform
#pragma unroll
            for (int t = 0; t < 3; ++t)
#pragma unroll
                for (int k = 0; k < kPer; ++k)
                    if (euse[k]) st[t * per + eidx[k]] = v[t][k];
        } else {
#pragma unroll
            for (int t = 0; t < 3; ++t)
#pragma unroll
                for (int k = 0; k < kPer; ++k) {
                    if (euse[k]) {
                        const bool ok = eidx[k] < valid;
                        c64 w;
                        w.re = ok ? v[t][k].re : 0.0;
                        w.im = ok ? v[t][k].im : 0.0;
                        st[t * per + eidx[k]] = w;
                    }
                }
        }
        __syncthreads();
        if (j0 + P < j_hi) load_stage(j0 + P);
        sk_tile_dispatch<NMAX>(nap, st, per, KP, P, nx, ay, ysg, kq, zc, are, aim);
    }

    // lane l: row 4 ((l / 4) % 4) + l / 16 of the tile, a = 2b + (l % 4) / 2,
    // component l % 2; the partner lane l ^ 1 holds the other z component
    const int r = tile_row0 + 4 * ((lane >> 2) & 3) + (lane >> 4);
    const int aoff = (lane >> 1) & 1, bim = lane & 1;
#pragma unroll
    for (int b = 0; b < NMAX; ++b) {
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

// Particles per staged sub-chunk: the largest of 48, 32, 16, 8 (a multiple of
// 8, two quads per step) whose three tables (3 P KP entries) fit kSmStage
// entries per thread.  0 if even 8 do not fit.
int sk_mfma_particles(int KP)
{
    static const int kCand[4] = {48, 32, 16, 8};
    for (int c = 0; c < 4; ++c)
        if (3 * kCand[c] * KP <= kSmStage * kSmWaves * kLanes) return kCand[c];
    return 0;
}

size_t sk_mfma_smem_bytes(int KP) { return (size_t)3 * sk_mfma_particles(KP) * KP * sizeof(c64); }

hipError_t launch_sk_mfma(hipStream_t s, const RecipArgs &a, int n_chunks, int chunk_len, const c64 *tx,
                          const c64 *ty, const c64 *tz, const int *row_nx, const int *row_ny, const int *row_m,
                          const int *unit_base, const int *tile_of, d4 *part)
{
    const int P = sk_mfma_particles(a.KP);
    const int n_rblocks = sk_mfma_row_blocks(a.n_rows);
    if (a.KP <= 2 * kSmNapSmall)
        hipLaunchKernelGGL(k_sk_mfma<kSmNapSmall>, dim3(xcd_grid(n_rblocks * n_chunks)), dim3(kSmWaves * kLanes),
                           sk_mfma_smem_bytes(a.KP), s, a.n, a.KP, P, a.n_rows, n_rblocks, n_chunks, chunk_len, tx, ty,
                           tz, row_nx, row_ny, row_m, unit_base, tile_of, a.n_slots, part);
    else
        hipLaunchKernelGGL(k_sk_mfma<kSmNap>, dim3(xcd_grid(n_rblocks * n_chunks)), dim3(kSmWaves * kLanes),
                           sk_mfma_smem_bytes(a.KP), s, a.n, a.KP, P, a.n_rows, n_rblocks, n_chunks, chunk_len, tx, ty,
                           tz, row_nx, row_ny, row_m, unit_base, tile_of, a.n_slots, part);
    return hipGetLastError();
}

}  // namespace ewk
