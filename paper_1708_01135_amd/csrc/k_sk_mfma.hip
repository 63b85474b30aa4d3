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
// y^n and z^n tables of P particles at a time in LDS (sk_mfma_particles),
// loading the next sub-chunk into a second buffer while it multiplies.  The
// partial sums of the chunk are written in the slot layout of the vector
// kernel (unit = (64-row group, a segment), a mod 8, row mod 64), so the same
// fixed-order reduction follows.
#include "ewald_internal.h"

namespace ewk {

namespace {

// Word 3 of a raw buffer resource on GFX9-family parts (32-bit data format,
// no swizzle); out-of-range loads return zero.
constexpr int kBufferWord3 = 0x00020000;
// s_waitcnt immediate with vmcnt = 0 and expcnt / lgkmcnt left at their
// maxima (GFX9 encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).
constexpr int kWaitVmcnt0 = 0x0F70;

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
__device__ __forceinline__ void sk_mfma_body(int bx, int by, int64_t n, int KP, int P, int n_rows, int n_rblocks,
                                             int n_chunks, int chunk_len, const c64 *__restrict__ tx,
                                             const c64 *__restrict__ ty, const c64 *__restrict__ tz,
                                             const int *__restrict__ row_nx, const int *__restrict__ row_ny,
                                             const int *__restrict__ row_m, const int *__restrict__ unit_base,
                                             const int *__restrict__ tile_of, int n_slots, d4 *__restrict__ part)
{
    extern __shared__ __align__(16) unsigned char smem[];  // two buffers of [3][P][KP]: q x^n, y^n, z^n
    const int nb = n_rblocks * n_chunks;
    const int bid = xcd_remap(bx, nb);
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

    // Staging, double-buffered: the three tables of a sub-chunk are each
    // per = P KP contiguous entries.  While the waves multiply sub-chunk i out
    // of one LDS buffer, the loads of sub-chunk i + 1 go straight from global
    // memory into the other (16-byte buffer loads to LDS: a wave's instruction
    // fills 64 consecutive entries, wave w taking entries 64 w + 512 k), with no
    // register round trip and no LDS store instructions.  Each table's buffer
    // resource ends at the sub-chunk's last particle, so the entries of a
    // partial sub-chunk (a chunk's last) past it load as zero.  The wait on the
    // wave's own loads (vmcnt) and the barrier at the top of each step make the
    // buffer complete before any wave reads it; the buffer the next loads
    // overwrite was last read before that barrier.
    constexpr int kStride = kSmWaves * kLanes;
    constexpr int kPer = kSmStage / 3;
    const int per = P * KP;
    c64 *const st = reinterpret_cast<c64 *>(smem);  // buffer b at st + 3 per b
    const c64 *tab[3] = {tx, ty, tz};
    const int wave_e0 = __builtin_amdgcn_readfirstlane(w * kLanes);
    auto stage = [&](int64_t j0, c64 *dst) {
        const int64_t left = j_hi - j0;
        const int valid = (left < P ? (int)left : P) * KP;  // entries of each table
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<c64 *>(tab[t] + j0 * KP), 0, valid * (int)sizeof(c64), kBufferWord3);
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const int e0 = wave_e0 + k * kStride;
                if (e0 < per && e0 + lane < per)
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(
                        rs, (__attribute__((address_space(3))) void *)(dst + t * per + e0), 16,
                        (e0 + lane) * (int)sizeof(c64), 0, 0, 0);
            }
        }
    };
    int cur = 0;
    if (j_lo < j_hi) stage(j_lo, st);
    for (int64_t j0 = j_lo; j0 < j_hi; j0 += P) {
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        __syncthreads();
        if (j0 + P < j_hi) stage(j0 + P, st + (cur ^ 1) * 3 * per);
        sk_tile_dispatch<NMAX>(nap, st + cur * 3 * per, per, KP, P, nx, ay, ysg, kq, zc, are, aim);
        cur ^= 1;
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

template <int NMAX>
struct KSkMfma {
    static constexpr int kThreads = kSmWaves *kLanes;
    static constexpr int kWavesPerEu = 2;
    int64_t n;
    int KP;
    int P;
    int n_rows;
    int n_rblocks;
    int n_chunks;
    int chunk_len;
    const c64 *tx;
    const c64 *ty;
    const c64 *tz;
    const int *row_nx;
    const int *row_ny;
    const int *row_m;
    const int *unit_base;
    const int *tile_of;
    int n_slots;
    d4 *part;
    __device__ void run(int bx, int by) const
    {
        sk_mfma_body<NMAX>(bx, by, n, KP, P, n_rows, n_rblocks, n_chunks, chunk_len, tx, ty, tz, row_nx, row_ny, row_m,
                           unit_base, tile_of, n_slots, part);
    }
    hipError_t one(hipStream_t s, dim3 grid, int threads, size_t smem) const;
};

template <int NMAX>
__global__ __launch_bounds__(kSmWaves *kLanes, 2) void k_sk_mfma(int64_t n, int KP, int P, int n_rows, int n_rblocks,
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
    sk_mfma_body<NMAX>(blockIdx.x, blockIdx.y, n, KP, P, n_rows, n_rblocks, n_chunks, chunk_len, tx, ty, tz, row_nx,
                       row_ny, row_m, unit_base, tile_of, n_slots, part);
}

template <int NMAX>
hipError_t KSkMfma<NMAX>::one(hipStream_t s, dim3 grid, int threads, size_t smem) const
{
    hipLaunchKernelGGL((k_sk_mfma<NMAX>), grid, dim3(threads), smem, s, n, KP, P, n_rows, n_rblocks, n_chunks,
                       chunk_len, tx, ty, tz, row_nx, row_ny, row_m, unit_base, tile_of, n_slots, part);
    return hipGetLastError();
}

}  // namespace

// Particles per staged sub-chunk (a multiple of 8: two quads per step).  The
// two buffers take 2 x 3 P KP entries of LDS, and the structure factor runs
// beside the real-space kernels, whose blocks need LDS on the same compute
// units: P is the largest of 48, 40, 32, 24, 16, 8 whose two buffers stay
// within 2 x 1792 entries (56 KiB; 2 x 2304, 72 KiB, beside the FP64
// real-space kernels, which hold fewer waves), as long as that P is at least
// 24; otherwise (large k_max) the largest P <= 32 whose tables fit kSmStage
// entries per thread, so that a step still holds enough quads to cover its
// barrier.  Measured: rock salt 32^3 (k_max 20) took 0.199 ms per mixed
// evaluation with P = 24, 0.204 with P = 32 and 0.211 with P = 48, and 0.257
// ms per FP64 evaluation with P = 32 against 0.267 with P = 24; rock salt
// 64^3 (k_max 32) 3.74 ms with P = 32 and 4.18 with P = 8.  0 if even 8
// particles do not fit.
int sk_mfma_particles(int KP, bool fp64)
{
    static const int kCand[6] = {48, 40, 32, 24, 16, 8};
    const int small_stage = fp64 ? 2304 : 1792;
    for (int c = 0; c < 6; ++c)
        if (3 * kCand[c] * KP <= small_stage) {
            if (kCand[c] >= 24) return kCand[c];
            break;
        }
    for (int c = 2; c < 6; ++c)
        if (3 * kCand[c] * KP <= kSmStage * kSmWaves * kLanes) return kCand[c];
    return 0;
}

size_t sk_mfma_smem_bytes(int KP, bool fp64)
{
    return (size_t)2 * 3 * sk_mfma_particles(KP, fp64) * KP * sizeof(c64);
}

hipError_t launch_sk_mfma(hipStream_t s, const RecipArgs &a, int n_chunks, int chunk_len, const c64 *tx,
                          const c64 *ty, const c64 *tz, const int *row_nx, const int *row_ny, const int *row_m,
                          const int *unit_base, const int *tile_of, d4 *part, bool fp64)
{
    const int P = sk_mfma_particles(a.KP, fp64);
    const int n_rblocks = sk_mfma_row_blocks(a.n_rows);
    const dim3 grid(xcd_grid(n_rblocks * n_chunks));
    if (a.KP <= 2 * kSmNapSmall)
        return launch(s, grid, kSmWaves * kLanes, sk_mfma_smem_bytes(a.KP, fp64),
                      KSkMfma<kSmNapSmall>{a.n, a.KP, P, a.n_rows, n_rblocks, n_chunks, chunk_len, tx, ty, tz, row_nx,
                                           row_ny, row_m, unit_base, tile_of, a.n_slots, part});
    return launch(s, grid, kSmWaves * kLanes, sk_mfma_smem_bytes(a.KP, fp64),
                  KSkMfma<kSmNap>{a.n, a.KP, P, a.n_rows, n_rblocks, n_chunks, chunk_len, tx, ty, tz, row_nx, row_ny,
                                  row_m, unit_base, tile_of, a.n_slots, part});
}

}  // namespace ewk
