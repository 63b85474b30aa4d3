// Internal declarations of the gfx950 Ewald library: plan layout, plain data
// types shared by the kernels and the host runtime, and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/ewald.h"

namespace ewk {

// Reciprocal-space work decomposition (see k_recip.hip):
//   a "row" is one (n_x, n_y) pair of the half space, carrying every n_z with
//   n_x^2 + n_y^2 + n_z^2 <= K^2, i.e. |n_z| <= m_row;
//   a "slot" is (row, a = |n_z|) and stands for the two vectors (n_x, n_y, +a) and
//   (n_x, n_y, -a), whose phases exp(+-i a theta_z) are complex conjugates;
//   a "segment" is a run of kQ consecutive a values (a = kQ*s ... kQ*s + kQ-1).
constexpr int kQ = 8;        // a values per segment
constexpr int kLanes = 64;   // wavefront width on CDNA
constexpr int kSkWaves = 4;  // waves per structure-factor block (one row group, one segment)

struct alignas(8) c32 {
    float re, im;
};
struct alignas(16) c64 {
    double re, im;
};
template <typename R>
struct Cplx;
template <>
struct Cplx<float> {
    using type = c32;
};
template <>
struct Cplx<double> {
    using type = c64;
};

// 32-byte record used for sorted particles (x, y, z, q), per-particle partial
// sums (phi, Fx, Fy, Fz) and structure-factor slots (S+ re, S+ im, S- re, S- im).
struct alignas(32) d4 {
    double a, b, c, d;
};

// Upper bound on the gather's k splits (grid.y) for small particle counts.
constexpr int kMaxSplit = 16;
struct SplitTable {
    int lo[kMaxSplit + 1];
};

enum KernelClass {
    KC_BIN = 0,
    KC_SCAN,
    KC_SCATTER,
    KC_CELLSORT,
    KC_PHASE,
    KC_SK,
    KC_SKREDUCE,
    KC_GATHER,
    KC_PAIRLIST,
    KC_PAIR,
    KC_FINAL_P,
    KC_FINAL_E,
    KC_COUNT
};
extern const char *const kKernelClassNames[KC_COUNT];

// ---- kernel launchers (each returns the hipGetLastError() of its launch) ----
struct CellArgs {
    int64_t n;
    double L;
    int nc;
    int ncell;
};
// Zero `bytes` (a multiple of 16, 16-byte aligned) at p with a fill kernel.
hipError_t launch_zero(hipStream_t s, void *p, size_t bytes);
hipError_t launch_bin(hipStream_t s, const CellArgs &a, const double *pos, const double *q, int *cell_of,
                      int *counts, double *qpart, int *status);
// Two launches: tile totals (and the charge sums), then the per-tile scans.
// tile_sums holds scan_tiles(ncell) entries.
int scan_tiles(int ncell);
hipError_t launch_scan(hipStream_t s, const CellArgs &a, int *counts, int *fill, int *cell_start,
                       const double *qpart, int n_qblocks, double *scalars, int2 *tile_sums, int *item_cell,
                       int *item_off, int *n_items);
hipError_t launch_scatter(hipStream_t s, const CellArgs &a, const int *cell_of, const int *cell_start,
                          int *fill, int *tmp_idx);
// One-workgroup cell list of a small system (n <= kSmallCellsMaxN, ncell <=
// kSmallCellsMaxCells): the outputs of bin, scan, scatter and cellsort, bit
// for bit (counts, fill and tile sums are not touched).  Measured on
// serving-mix electrolytes: 0.090 against 0.095 ms per call at 256 ions, even
// at 512, 0.19 against 0.10 at 2048 (one workgroup's O(n^2) ranks and serial
// chunks lose to the spread kernels).
constexpr int kSmallCellsMaxN = 512;
constexpr int kSmallCellsMaxCells = 4096;
bool cells_small(const CellArgs &a);
hipError_t launch_cells_small(hipStream_t s, const CellArgs &a, const double *pos, const double *q, int *cell_start,
                              int *item_cell, int *item_off, int *n_items, double *scalars, int *perm, d4 *pq,
                              int *status);
hipError_t launch_cellsort(hipStream_t s, const CellArgs &a, const int *cell_start, int *tmp_idx,
                           const double *pos, const double *q, int *perm, d4 *pq);

struct RecipArgs {
    int64_t n;
    double L;
    int K;        // k_max
    int KP;       // padded per-particle table length (multiple of kQ, >= K+1)
    int n_rows;
    int n_units;
    int n_items;
    int n_slots;  // n_units * kQ * kLanes
};
// Phase tables in caller order from the caller's positions and charges; also
// writes pr[j] = (wrapped x, y, z, q), the particle records of the reciprocal
// kernels (which therefore do not wait for the cell list).
template <typename R>
hipError_t launch_phase(hipStream_t s, const RecipArgs &a, const double *pos, const double *q, d4 *pr,
                        typename Cplx<R>::type *tx, typename Cplx<R>::type *ty, typename Cplx<R>::type *tz);
// table rows per phase block for a KP (fewer when the LDS stage would pass 64 KB)
template <typename R>
int phase_rows(int KP);
// lanes per slot in the structure-factor reduction (k_sk_reduce)
constexpr int kRedSlotLanes = 4;
// structure factor (FP64 phases and sums in both precisions)
size_t sk_smem_bytes(int ts, int K1);
int sk_tile(int K1);
hipError_t launch_sk(hipStream_t s, const RecipArgs &a, int n_chunks, int chunk_len, const c64 *tx, const c64 *ty,
                     const c64 *tz, const int *unit_group, const int *unit_seg, const int *row_nx, const int *row_ny,
                     d4 *part);
// Matrix-core gather (k_gather_mfma.hip).  The half-space rows are cut, along
// each n_x line, into quads of kMQuad consecutive n_y; quads sorted by their
// largest m are grouped kMTileQuads to a tile of 16 rows (the M dimension of a
// 16x16x4 MFMA).  A tile's coefficients are stored per pair of |n_z| values
// (a = 2p, 2p+1) as one block of kMBlock values [quantity 4][k 4][row 16]:
// quantities T_re, T_im, Tz_re, Tz_im; k = (Re z^a, Im z^a, Re z^(a+1),
// Im z^(a+1)); row = 4 * quad + offset in the quad (FP32), or 4 * offset + quad
// (FP64, whose MFMA interleaves its output rows over the lane groups).
constexpr int kMQuad = 4;
constexpr int kMTileQuads = 4;
constexpr int kMBlock = 256;
struct MTile {
    int base;     // first coefficient block of the tile
    int nap;      // a pairs (ceil((m_max + 1) / 2))
    int quad[kMTileQuads];  // n_x << 16 | (n_y of the quad's first row + 32768)
};
// sk_reduce writes the VALU gather records to `rec` and, when `mcoef` is
// given, the same coefficients in the tile layout at row_mbase[row] +
// (a >> 1) * kMBlock + q * 64 + ((a & 1) * 2 + c) * 16 (c = 0: factor of
// Re z^a, c = 1: of Im z^a).
template <typename R>
hipError_t launch_sk_reduce(hipStream_t s, const RecipArgs &a, int n_chunks, const d4 *part,
                            const int *unit_group, const int *unit_seg, const int *row_nx,
                            const int *row_ny, const int *row_m, const int *row_item, const double *ck,
                            d4 *sk, R *rec, R *mcoef, const int *row_mbase, double *erec_part);
// Matrix-core structure factor (k_sk_mfma.hip): one block per (128 rows,
// particle chunk), one wave per 16-row tile holding up to kSmNap pairs of a
// values in FP64 MFMA accumulators (k_max <= 2 kSmNap - 1).
constexpr int kSmWaves = kLanes / 8;
constexpr int kSmTileRows = 16;
constexpr int kSmNap = 24;
constexpr int kSmNapSmall = 12;  // the instance for KP <= 2 kSmNapSmall
constexpr int kSmMaxKP = 2 * kSmNap;  // k_max + 1 <= KP <= kSmMaxKP
constexpr int kSmStage = 9;  // staged entries per thread and buffer, a multiple of 3: 3 P KP <= kSmStage * kSmWaves * kLanes
// (fp64: the plan's precision, which sets how much LDS the real-space kernels
// beside it leave)
int sk_mfma_particles(int KP, bool fp64);
size_t sk_mfma_smem_bytes(int KP, bool fp64);
inline int sk_mfma_row_blocks(int n_rows) { return (n_rows + kSmWaves * kSmTileRows - 1) / (kSmWaves * kSmTileRows); }
// tile_of[block * kSmWaves + w]: the 16-row tile of wave w in row block `block`, or -1.
hipError_t launch_sk_mfma(hipStream_t s, const RecipArgs &a, int n_chunks, int chunk_len, const c64 *tx,
                          const c64 *ty, const c64 *tz, const int *row_nx, const int *row_ny, const int *row_m,
                          const int *unit_base, const int *tile_of, d4 *part, bool fp64);
// Particles per block of the matrix-core gather (16 per sub-tile): 32, or in
// FP32 64 from 65536 particles on.  A block streams every coefficient of its
// row split once, so 64 halves that traffic; below 65536 particles the
// 32-particle blocks' higher occupancy wins (measured: rock salt 32^3 took
// 0.225 ms per evaluation with 64 against 0.210 with 32; 64^3 3.70 against
// 3.75-3.80 ms).
constexpr int64_t kGatherWideFrom = 65536;
inline int gather_mfma_particles(int64_t n, bool fp64) { return !fp64 && n >= kGatherWideFrom ? 64 : 32; }
// LDS of the z-power stage alone, and of the whole matrix-core gather block
// (stage and phase tables, or the cross-wave sums if larger), for blocks of np
// particles.
size_t gather_mfma_stage_bytes(int nap_max, int np, bool fp64);
size_t gather_mfma_smem_bytes(int nap_max, int np, int K, bool fp64);
template <typename R>
hipError_t launch_gather_mfma(hipStream_t s, const RecipArgs &a, int n_split, const SplitTable &split, int nap_max,
                              const d4 *pq, const c64 *tz, const MTile *tiles, const R *mcoef, d4 *gpart);
// gather items carry a packed word: segment << 16 | n_x << 8 | (n_y + 128)
template <typename R>
hipError_t launch_gather(hipStream_t s, const RecipArgs &a, int n_split, const SplitTable &split,
                         const d4 *pq, const c64 *tz, const int *item_meta, const R *rec, d4 *gpart);

struct PairArgs {
    int64_t n;
    double L;
    int nc;
    int ncell;
    double rc2;
    double alpha;
};
// Real-space cells have side >= r_c / kPairReach, so the stencil spans
// (2 kPairReach + 1)^3 cells.  Neighbour lists hold 32-bit entries: the sorted
// index j in the low kPairIndexBits bits and the image-shift code above them;
// particle i's list is list[i * cap ...].  List-building work items are (cell,
// kPairHome consecutive home particles).
constexpr int kPairReach = 2;
constexpr int kPairHome = 8;
constexpr int kPairIndexBits = 25;
constexpr int64_t kPairMaxN = (int64_t)1 << kPairIndexBits;  // largest n_max the lists can index
// Small systems, whose work items would leave the chip mostly idle, spread
// each item's home particles over up to kPairHome waves in the list pass
// (pair_list_split: the smallest power of two that gives kPairSmallWaves
// waves), and give each particle a whole wave in the evaluation pass when
// fewer than kPairSmallWaves / 2 waves of kPairHome particles would run
// (pair_small).  Lists are the same either way.
constexpr int kPairSmallWaves = 2048;
int pair_list_split(int max_items);
bool pair_small(int64_t n);
hipError_t launch_pair_list(hipStream_t s, const PairArgs &a, int max_items, const int *n_items,
                            const int *item_cell, const int *item_off, const int *cell_start, const d4 *pq,
                            uint32_t *list, int *list_cnt, int cap);
hipError_t launch_pair(hipStream_t s, const PairArgs &a, bool mixed, const int *cell_start, const d4 *pq,
                       const uint32_t *list, const int *list_cnt, int cap, d4 *freal);

struct FinalArgs {
    int64_t n;
    double L;
    double alpha;
    int n_split;           // gather partials to sum (0: energy only)
    int n_erec;
    const double *gscale;  // device scalar g (or null): forces := -g F, dEdq := g dE/dq
};
// freal, pq are in cell-sorted order; gpart (reciprocal partial sums) in caller
// order, read through perm.
hipError_t launch_finalize_particles(hipStream_t s, const FinalArgs &a, const d4 *pq, const int *perm,
                                     const d4 *freal, const d4 *gpart, const double *scalars,
                                     double *forces, double *dEdq, double *epart);
// Both totals passes in one workgroup for a small system (n <= 512), with the
// same sums in the same order as launch_finalize_particles + _energy.
bool finalize_small(int64_t n);
hipError_t launch_finalize_small(hipStream_t s, const FinalArgs &a, const d4 *pq, const int *perm, const d4 *freal,
                                 const d4 *gpart, const double *scalars, double *forces, double *dEdq,
                                 const double *erec_part, const int *status, double *energy);
hipError_t launch_finalize_energy(hipStream_t s, const FinalArgs &a, const double *epart, int n_epart,
                                  const double *erec_part, const double *scalars, const int *status,
                                  double *energy);

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// ---- one launch per system, or one launch for many systems ----
// Every kernel is a plain struct of its arguments with
//   static constexpr int kThreads;               block size
//   static constexpr int kWavesPerEu;            waves per SIMD the registers must allow (1: no bound)
//   __device__ void run(int bx, int by) const;   the work of block (bx, by)
//   hipError_t one(stream, grid, threads, smem) const;
//                                                launch of a plain kernel, with the
//                                                same parameters, that calls the same code
// one() keeps the parameters as kernel arguments, whose no-alias
// qualifiers let the compiler turn uniform loads into scalar ones; a
// pointer read from a struct would lose that.  k_many runs the structs of up to
// BatchPack<K>::kCap systems in one 1-D grid over a ragged work list: system s
// owns the blocks [span[s].first, span[s + 1].first), laid out gx = span[s].gx
// wide, and block b of the launch runs block ((b - first) % gx, (b - first) /
// gx) of its system.  The structs travel in the kernel arguments (at most
// kBatchKernargBytes), so a batch needs no device memory and no copy of its
// own.  Both kernels run the same body, so a system's results do not depend
// on which launch ran it.
struct BatchSpan {
    int first;
    int gx;
};
constexpr size_t kBatchKernargBytes = 4096;

template <class K>
struct BatchPack {
    static constexpr int kCap = (int)((kBatchKernargBytes - 2 * sizeof(BatchSpan) - 8) / (sizeof(K) + sizeof(BatchSpan)));
    K ks[kCap];
    BatchSpan span[kCap + 1];
    int nsys;
};

template <class K>
__global__ __attribute__((amdgpu_flat_work_group_size(1, K::kThreads), amdgpu_waves_per_eu(K::kWavesPerEu))) void
k_many(BatchPack<K> pk)
{
    const int b = (int)blockIdx.x;
    int lo = 0, hi = pk.nsys;  // span[lo].first <= b < span[hi].first
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pk.span[mid].first <= b)
            lo = mid;
        else
            hi = mid;
    }
    const int local = b - pk.span[lo].first, gx = pk.span[lo].gx;
    pk.ks[lo].run(local % gx, local / gx);
}

// A launch held for a batch instead of being enqueued (see BatchRecorder), and
// the layout of its kernel's BatchPack.
struct LaunchRecord {
    const void *many;   // host stub of k_many<K>
    int threads;
    dim3 grid;
    size_t smem;
    size_t args_off;    // K's bytes in BatchRecorder::args
    size_t args_size;   // sizeof(K)
    int cap;            // BatchPack<K>::kCap
    size_t span_off, nsys_off, pack_size;
    int kind;           // rank of the launch's kernel class in the launch order
    int occ;            // earlier launches of this system in the same class
    int sys;
};
// While a host thread has a recorder installed (batch evaluation), launch()
// appends to it instead of launching.
struct BatchRecorder {
    std::vector<LaunchRecord> recs;
    std::vector<unsigned char> args;
    int kind = 0;
    int sys = 0;
    int occ = 0;
    void add(const LaunchRecord &r, const void *k);
};
extern thread_local BatchRecorder *t_batch;

// threads: the block size, at most K::kThreads
template <class K>
hipError_t launch(hipStream_t s, dim3 grid, int threads, size_t smem, const K &k)
{
    static_assert(std::is_trivially_copyable<K>::value, "kernel arguments are copied as bytes");
    using Pack = BatchPack<K>;
    static_assert(Pack::kCap >= 8 && sizeof(Pack) <= kBatchKernargBytes, "batch pack");
    if (t_batch) {
        LaunchRecord r{};
        r.many = reinterpret_cast<const void *>(&k_many<K>);
        r.threads = threads;
        r.grid = grid;
        r.smem = smem;
        r.args_size = sizeof(K);
        r.cap = Pack::kCap;
        r.span_off = offsetof(Pack, span);
        r.nsys_off = offsetof(Pack, nsys);
        r.pack_size = sizeof(Pack);
        t_batch->add(r, &k);
        return hipSuccess;
    }
    return k.one(s, grid, threads, smem);
}

// Position reduced into [0, L) (NaN and infinities map to 0; they are flagged
// separately).  Shared by the cell binning and the phase tables so that both
// halves of the evaluation see the same wrapped coordinates.
__device__ inline double wrap_coord(double x, double L)
{
    double w = x - L * floor(x / L);
    if (w < 0.0) w += L;
    if (w >= L) w -= L;
    if (!(w >= 0.0 && w < L)) w = 0.0;  // also catches NaN
    return w;
}

// MI355X dispatches the workgroups of a launch to its 8 XCDs round-robin by
// linear block id, and each XCD has its own L2.  Kernels whose neighbouring
// work items share data launch xcd_grid(n) blocks and map the hardware id
// through xcd_remap(), which gives every XCD a contiguous range of logical
// blocks; logical ids >= n are padding and exit at once.
constexpr int kXcds = 8;
inline int xcd_grid(int n) { return ceil_div(n, kXcds) * kXcds; }
__device__ inline int xcd_remap(int b, int n)
{
    const int per = (n + kXcds - 1) / kXcds;
    return (b % kXcds) * per + b / kXcds;
}

}  // namespace ewk
