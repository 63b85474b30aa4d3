// Host runtime of the C ABI declared in include/ewald.h: parameter checks,
// plan-time tables (k-set layout, C_k, cell grid), one device allocation for
// all workspace, and the per-call launch sequence on the plan's stream.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "ewald_internal.h"

using namespace ewk;

namespace ewk {
const char *const kKernelClassNames[KC_COUNT] = {"bin",    "scan",   "scatter",  "cellsort", "phase",  "sk",
                                                 "sk_reduce", "gather", "pair_list", "pair", "final_p", "final_e"};
int bin_blocks(int64_t n);

thread_local BatchRecorder *t_batch = nullptr;

void BatchRecorder::add(const LaunchRecord &rec, const void *k)
{
    LaunchRecord r = rec;
    r.args_off = args.size();
    r.kind = kind;
    r.occ = occ++;
    r.sys = sys;
    const unsigned char *b = static_cast<const unsigned char *>(k);
    args.insert(args.end(), b, b + r.args_size);
    recs.push_back(r);
}
}  // namespace ewk

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr int kMaxCellsPerAxis = 128;
constexpr int kSkTargetBlocks = 2048;     // structure-factor blocks wanted in flight
constexpr int kGatherTargetBlocks = 1024; // gather blocks wanted in flight
constexpr int kMaxChunks = 1024;

// ---------------------------------------------------------- k-set layout
struct KLayout {
    int K = 0, KP = 0;
    int n_rows = 0, n_units = 0, n_items = 0, n_segmax = 0;
    int64_t kcount = 0;
    // rows sorted by m (descending): structure-factor lanes
    std::vector<int> row_nx, row_ny, row_m;
    std::vector<int> unit_g, unit_s;
    // gather items: per segment, rows with m >= kQ*s in (nx, ny) order
    std::vector<int> item_nx, item_ny, item_seg;
    std::vector<int> item_meta;  // seg << 16 | nx << 8 | (ny + 128)
    std::vector<int> row_item;   // [seg * n_rows + row] -> item, or -1
    // matrix-core gather: tiles of kMTileQuads quads (kMQuad consecutive n_y at one n_x)
    std::vector<MTile> mtiles;
    std::vector<int> row_mbase;      // per (sorted) row: offset of its (tile, row) coefficients
    std::vector<int64_t> nap_prefix; // prefix sums of the tiles' a pairs
    int m_blocks = 0, nap_max = 0;
    std::vector<int> unit_base;      // first structure-factor unit of each 64-row group
    std::vector<int> sk_tile_of;     // matrix-core structure factor: tile of (row block, wave), or -1
};

int isqrt_floor(int v)
{
    int r = (int)std::floor(std::sqrt((double)v));
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

// Tiles of the matrix-core structure factor dealt to (row block, wave).  Tiles
// (16 rows in the structure-factor order) are sorted by their pairs of a,
// heaviest first.  Waves w and w + 4 of a block
// share a SIMD: the i-th heaviest tile is paired with the i-th lightest (slots
// past the last tile are empty), and the pairs are dealt round-robin over the
// row blocks, so every block's busiest SIMD carries about the average load.
void build_sk_tiles(KLayout &kl)
{
    const int rows_per_tile = kSmTileRows;
    const int n_tiles = (kl.n_rows + rows_per_tile - 1) / rows_per_tile;
    const int n_rb = (n_tiles + kSmWaves - 1) / kSmWaves;
    const int slots = n_rb * kSmWaves;
    const int half = kSmWaves / 2;
    kl.sk_tile_of.assign(slots, -1);
    for (int pr = 0; pr < slots / 2; ++pr) {
        const int heavy = pr, light = slots - 1 - pr;
        const int blk = pr % n_rb, k = pr / n_rb;  // k-th pair of block blk: waves k and k + half
        kl.sk_tile_of[blk * kSmWaves + k] = heavy < n_tiles ? heavy : -1;
        kl.sk_tile_of[blk * kSmWaves + k + half] = light < n_tiles ? light : -1;
    }
}

// fp64_rows: the FP64 16x16x4 MFMA returns row 4 r + g of its output in lane
// group g, register r (the FP32 one returns row 4 g + r); the tile rows of a
// quad's n_y offsets follow the instruction the plan will use, so that lane
// group g always holds quad g.
void build_klayout(int K, KLayout &kl, bool fp64_rows = false)
{
    kl.K = K;
    kl.KP = ((K + 1 + kQ - 1) / kQ) * kQ;
    struct Row {
        int nx, ny, m;
    };
    std::vector<Row> nat;  // natural (nx, ny) order of the half space
    const int K2 = K * K;
    nat.push_back({0, 0, K});
    for (int ny = 1; ny <= K; ++ny) nat.push_back({0, ny, isqrt_floor(K2 - ny * ny)});
    for (int nx = 1; nx <= K; ++nx) {
        const int M = isqrt_floor(K2 - nx * nx);
        for (int ny = -M; ny <= M; ++ny) nat.push_back({nx, ny, isqrt_floor(K2 - nx * nx - ny * ny)});
    }
    kl.n_rows = (int)nat.size();
    kl.kcount = 0;
    for (const Row &r : nat) kl.kcount += (r.nx == 0 && r.ny == 0) ? r.m : 2 * r.m + 1;

    std::vector<int> order(nat.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nat[a].m > nat[b].m; });
    std::vector<int> sorted_of_nat(nat.size());
    kl.row_nx.resize(nat.size());
    kl.row_ny.resize(nat.size());
    kl.row_m.resize(nat.size());
    for (size_t r = 0; r < order.size(); ++r) {
        const Row &w = nat[order[r]];
        kl.row_nx[r] = w.nx;
        kl.row_ny[r] = w.ny;
        kl.row_m[r] = w.m;
        sorted_of_nat[order[r]] = (int)r;
    }
    kl.n_segmax = K / kQ + 1;
    const int n_groups = (kl.n_rows + kLanes - 1) / kLanes;
    kl.unit_g.clear();
    kl.unit_s.clear();
    for (int g = 0; g < n_groups; ++g) {
        const int mmax = kl.row_m[g * kLanes];
        for (int s = 0; s <= mmax / kQ; ++s) {
            kl.unit_g.push_back(g);
            kl.unit_s.push_back(s);
        }
    }
    kl.n_units = (int)kl.unit_g.size();
    kl.unit_base.assign(n_groups, 0);
    for (int u = kl.n_units - 1; u >= 0; --u) kl.unit_base[kl.unit_g[u]] = u;
    kl.row_item.assign((size_t)kl.n_segmax * kl.n_rows, -1);
    kl.item_nx.clear();
    kl.item_ny.clear();
    kl.item_seg.clear();
    for (int s = 0; s < kl.n_segmax; ++s)
        for (size_t i = 0; i < nat.size(); ++i) {
            if (nat[i].m < s * kQ) continue;
            kl.row_item[(size_t)s * kl.n_rows + sorted_of_nat[i]] = (int)kl.item_nx.size();
            kl.item_nx.push_back(nat[i].nx);
            kl.item_ny.push_back(nat[i].ny);
            kl.item_seg.push_back(s);
        }
    kl.n_items = (int)kl.item_nx.size();
    kl.item_meta.resize(kl.n_items);
    for (int i = 0; i < kl.n_items; ++i)
        kl.item_meta[i] = (kl.item_seg[i] << 16) | (kl.item_nx[i] << 8) | (kl.item_ny[i] + 128);

    // Matrix-core tiles.  Each n_x line of the natural order (n_y consecutive) is
    // cut into quads; quads are sorted by their largest m (stable) and grouped
    // into tiles, the last one padded with empty quads (zero coefficients).
    struct Quad {
        int nx, ny0, m;
        size_t first, count;
    };
    std::vector<Quad> quads;
    for (size_t i = 0; i < nat.size();) {
        size_t e = i;
        while (e < nat.size() && nat[e].nx == nat[i].nx) ++e;
        for (size_t b = i; b < e; b += kMQuad) {
            Quad q{nat[b].nx, nat[b].ny, -1, b, std::min<size_t>(kMQuad, e - b)};
            for (size_t u = b; u < b + q.count; ++u) q.m = std::max(q.m, nat[u].m);
            quads.push_back(q);
        }
        i = e;
    }
    std::stable_sort(quads.begin(), quads.end(), [](const Quad &a, const Quad &b) { return a.m > b.m; });
    kl.mtiles.clear();
    kl.row_mbase.assign(nat.size(), 0);
    kl.nap_prefix.assign(1, 0);
    kl.m_blocks = 0;
    kl.nap_max = 0;
    for (size_t t0 = 0; t0 < quads.size(); t0 += kMTileQuads) {
        MTile tl{};
        tl.base = kl.m_blocks;
        tl.nap = (quads[t0].m + 2) / 2;  // a = 0 .. m in pairs
        for (int g = 0; g < kMTileQuads; ++g) {
            tl.quad[g] = 32768;  // empty quad: n_x = n_y = 0, no coefficients
            if (t0 + g >= quads.size()) continue;
            const Quad &q = quads[t0 + g];
            tl.quad[g] = (q.nx << 16) | (q.ny0 + 32768);
            for (size_t u = 0; u < q.count; ++u)
                kl.row_mbase[sorted_of_nat[q.first + u]] =
                    tl.base * kMBlock + (fp64_rows ? (int)u * kMTileQuads + g : g * kMQuad + (int)u);
        }
        kl.m_blocks += tl.nap;
        kl.nap_max = std::max(kl.nap_max, tl.nap);
        kl.nap_prefix.push_back(kl.nap_prefix.back() + tl.nap);
        kl.mtiles.push_back(tl);
    }
    build_sk_tiles(kl);
}

// Cells per axis for the pair loop: side h = L / nc >= r_c / kPairReach.
int cells_per_axis(double L, double rc)
{
    const double f = std::floor(kPairReach * L / rc);
    int nc = f < 1.0 ? 1 : (f > kMaxCellsPerAxis ? kMaxCellsPerAxis : (int)f);
    // guard against rounding just above an integer: h * kPairReach must stay >= rc
    while (nc > 1 && (L / nc) * kPairReach < rc) --nc;
    return nc;
}

int sk_chunks(int64_t n, int n_units, int tile)
{
    // at least one tile per wave of a block
    const int64_t by_work = (n + (int64_t)tile * kSkWaves - 1) / ((int64_t)tile * kSkWaves);
    int64_t want = (kSkTargetBlocks + n_units - 1) / n_units;
    if (want < 1) want = 1;
    int64_t c = std::min<int64_t>(by_work, want);
    c = std::min<int64_t>(c, kMaxChunks);
    return (int)std::max<int64_t>(c, 1);
}

int gather_split(int64_t n)
{
    const int64_t blocks = (n + 255) / 256;
    int64_t s = (kGatherTargetBlocks + blocks - 1) / blocks;
    return (int)std::min<int64_t>(std::max<int64_t>(s, 1), kMaxSplit);
}

// Row splits (grid.y) of the matrix-core gather: enough blocks to fill the
// chip, at least two tiles per wave on average; split boundaries balance the
// tiles' a pairs.
constexpr int kMfmaTargetBlocks = 1024;
// Blocks of kSmWaves waves in one round over the 256 CUs: one per CU.  The
// structure factor runs beside the real-space kernels, and one block per CU
// left them more of each SIMD: rock salt 32^3 (k_max 20) took 0.218 instead of
// 0.223 ms per evaluation with two.
constexpr int kSkMfmaBlocksPerCu = 1;
int sk_mfma_target_blocks() { return 256 * kSkMfmaBlocksPerCu; }

// Particle chunks the matrix-core structure factor may use (partial-sum capacity).
int sk_mfma_chunk_cap(const KLayout &kl)
{
    return std::max(1, std::min(kMaxChunks, sk_mfma_target_blocks() / sk_mfma_row_blocks(kl.n_rows)));
}

int gather_mfma_split(int64_t n, const KLayout &kl, bool fp64)
{
    const int np = gather_mfma_particles(n, fp64);
    const int64_t blocks = (n + np - 1) / np;
    int64_t s = (kMfmaTargetBlocks + blocks - 1) / blocks;
    s = std::min<int64_t>(s, (int64_t)kl.mtiles.size() / 8);
    return (int)std::min<int64_t>(std::max<int64_t>(s, 1), kMaxSplit);
}

void mfma_split_table(const KLayout &kl, int n_split, SplitTable &st)
{
    const int64_t tot = kl.nap_prefix.back();
    size_t t = 0;
    st.lo[0] = 0;
    for (int k = 1; k < n_split; ++k) {
        const int64_t want = tot * k / n_split;
        while (t < kl.mtiles.size() && kl.nap_prefix[t] < want) ++t;
        st.lo[k] = (int)t;
    }
    st.lo[n_split] = (int)kl.mtiles.size();
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Sizes of every device buffer; shared by the admission query, the plan and
// the static-scratch evaluation.  "Tables" are the plan's constants and its
// status word; the "work" buffers are what one evaluation of up to N particles
// writes and reads.
struct Sizes {
    size_t cell_of, counts, fill, cell_start, tmp_idx, perm, status;
    size_t pq, freal, qpart, scalars, epart, erec, ck;
    size_t tx, part, sk, rec, gpart;
    size_t row_nx, row_ny, row_m, unit_g, unit_s, row_item, item_nx, item_ny, item_seg;
    size_t pitem_cell, pitem_off, n_pitems, plist, plist_cnt, tile_sums;
    size_t mcoef, mtiles, row_mbase, unit_base, sk_tile_of, pr;
    size_t tables, work, total;
    int max_chunks;
    int max_pitems;  // pair work items: cells + n/kPairHome bounds sum_c ceil(count_c / kPairHome)
    int list_cap;    // neighbour-list entries per particle
};

// Neighbour-list capacity: 1.5x the expected count inside r_c at the plan's
// largest density, plus slack; lanes beyond it fall back to the direct loop.
int pair_list_cap(const ewald_params &p)
{
    const double rho = (double)p.n_max / (p.box_L * p.box_L * p.box_L);
    const double expect = 4.0 / 3.0 * kPi * p.r_c * p.r_c * p.r_c * rho;
    double cap = 1.5 * expect + 32.0;
    cap = std::min(cap, (double)p.n_max * 27.0 + 32.0);
    return (int)std::min(cap, 60000.0);
}

// N: particles the work buffers are sized for (n_max for a plan's own
// workspace, the call's n for the static scratch).
void compute_sizes(const ewald_params &p, const KLayout &kl, int nc, int64_t N, Sizes &z)
{
    const bool mixed = p.precision == EWALD_PRECISION_MIXED;
    const size_t ncell = (size_t)nc * nc * nc;
    const size_t creal = sizeof(c64);  // phase tables are FP64 in both precisions
    const size_t real = mixed ? sizeof(float) : sizeof(double);
    const int tile = sk_tile(kl.K + 1);
    z.max_chunks = std::max(sk_chunks(N, kl.n_units, tile), sk_mfma_chunk_cap(kl));
    const size_t n_slots = (size_t)kl.n_units * kQ * kLanes;
    const size_t gcap = std::min<size_t>((size_t)kMaxSplit * N, (size_t)kGatherTargetBlocks * 256 + N);
    z.cell_of = align_up(sizeof(int) * N);
    z.counts = align_up(sizeof(int) * ncell);
    z.fill = align_up(sizeof(int) * ncell);
    z.cell_start = align_up(sizeof(int) * (ncell + 1));
    z.tmp_idx = align_up(sizeof(int) * N);
    z.perm = align_up(sizeof(int) * N);
    z.status = align_up(sizeof(int) * 2);
    z.pq = align_up(sizeof(d4) * N);
    z.freal = align_up(sizeof(d4) * N);
    z.qpart = align_up(sizeof(double) * 2 * (size_t)bin_blocks(N));
    z.scalars = align_up(sizeof(double) * 4);
    z.epart = align_up(sizeof(double) * (size_t)ceil_div(N, 256));
    z.erec = align_up(sizeof(double) * (size_t)ceil_div((int64_t)n_slots, 256 / kRedSlotLanes));
    z.ck = align_up(sizeof(double) * ((size_t)kl.K * kl.K + 1));
    z.tx = align_up(creal * (size_t)N * kl.KP);
    z.part = align_up(sizeof(d4) * (size_t)z.max_chunks * n_slots);
    z.sk = align_up(sizeof(d4) * n_slots);
    z.rec = align_up(real * (size_t)kl.n_items * kQ * 8);
    z.gpart = align_up(sizeof(d4) * gcap);
    z.row_nx = z.row_ny = z.row_m = align_up(sizeof(int) * kl.n_rows);
    z.unit_g = z.unit_s = align_up(sizeof(int) * kl.n_units);
    z.row_item = align_up(sizeof(int) * kl.row_item.size());
    z.item_nx = z.item_ny = z.item_seg = align_up(sizeof(int) * (size_t)std::max(kl.n_items, 1));
    z.max_pitems = (int)ncell + ceil_div(N, kPairHome);
    z.pitem_cell = z.pitem_off = align_up(sizeof(int) * (size_t)z.max_pitems);
    z.n_pitems = align_up(sizeof(int));
    z.tile_sums = align_up(sizeof(int2) * (size_t)scan_tiles((int)ncell));
    z.list_cap = pair_list_cap(p);
    z.plist = align_up(sizeof(uint32_t) * (size_t)z.list_cap * N);
    z.plist_cnt = align_up(sizeof(int) * N);
    z.mcoef = align_up(real * (size_t)kl.m_blocks * kMBlock);
    z.mtiles = align_up(sizeof(MTile) * kl.mtiles.size());
    z.row_mbase = align_up(sizeof(int) * (size_t)kl.n_rows);
    z.unit_base = align_up(sizeof(int) * kl.unit_base.size());
    z.sk_tile_of = align_up(sizeof(int) * kl.sk_tile_of.size());
    z.pr = align_up(sizeof(d4) * N);
    z.tables = z.status + z.ck + 3 * z.row_nx + 2 * z.unit_g + z.row_item + 3 * z.item_nx + z.mtiles + z.row_mbase +
               z.unit_base + z.sk_tile_of;
    z.work = z.cell_of + z.counts + z.fill + z.cell_start + z.tmp_idx + z.perm + z.pq + z.freal + z.qpart +
             z.scalars + z.epart + z.erec + 3 * z.tx + z.part + z.sk + z.rec + z.gpart + 2 * z.pitem_cell +
             z.n_pitems + z.plist + z.plist_cnt + z.mcoef + z.pr + z.tile_sums;
    z.total = z.tables + z.work;
}

// Per-evaluation buffers, carved from the plan's allocation or from the
// static scratch.
struct Work {
    int *cell_of = nullptr, *counts = nullptr, *fill = nullptr, *cell_start = nullptr, *tmp_idx = nullptr,
        *perm = nullptr;
    d4 *pq = nullptr, *freal = nullptr, *part = nullptr, *sk = nullptr, *gpart = nullptr;
    double *qpart = nullptr, *scalars = nullptr, *epart = nullptr, *erec = nullptr;
    void *tx = nullptr, *ty = nullptr, *tz = nullptr, *rec = nullptr;
    int *pitem_cell = nullptr, *pitem_off = nullptr, *n_pitems = nullptr, *plist_cnt = nullptr;
    uint32_t *plist = nullptr;
    void *mcoef = nullptr;
    d4 *pr = nullptr;  // caller-order particle records of the reciprocal kernels
    int2 *tile_sums = nullptr;  // cell-scan tile totals
    int max_chunks = 1, list_cap = 1;
};

template <typename T>
T *carve(char *&cur, size_t bytes)
{
    T *r = reinterpret_cast<T *>(cur);
    cur += bytes;
    return r;
}

// The buffers that must hold zeros when an evaluation starts come first, so
// that one fill clears them: the cell counters (each evaluation leaves them
// cleared again) and the tile coefficients, whose padding entries are never
// written.
size_t zeroed_bytes(const Sizes &z) { return z.counts + z.fill + z.mcoef; }

void carve_work(char *cur, const Sizes &z, Work &w)
{
    w.counts = carve<int>(cur, z.counts);
    w.fill = carve<int>(cur, z.fill);
    w.mcoef = carve<void>(cur, z.mcoef);
    w.cell_of = carve<int>(cur, z.cell_of);
    w.cell_start = carve<int>(cur, z.cell_start);
    w.tmp_idx = carve<int>(cur, z.tmp_idx);
    w.perm = carve<int>(cur, z.perm);
    w.pq = carve<d4>(cur, z.pq);
    w.freal = carve<d4>(cur, z.freal);
    w.qpart = carve<double>(cur, z.qpart);
    w.scalars = carve<double>(cur, z.scalars);
    w.epart = carve<double>(cur, z.epart);
    w.erec = carve<double>(cur, z.erec);
    w.tx = carve<void>(cur, z.tx);
    w.ty = carve<void>(cur, z.tx);
    w.tz = carve<void>(cur, z.tx);
    w.part = carve<d4>(cur, z.part);
    w.sk = carve<d4>(cur, z.sk);
    w.rec = carve<void>(cur, z.rec);
    w.gpart = carve<d4>(cur, z.gpart);
    w.pitem_cell = carve<int>(cur, z.pitem_cell);
    w.pitem_off = carve<int>(cur, z.pitem_off);
    w.n_pitems = carve<int>(cur, z.n_pitems);
    w.plist = carve<uint32_t>(cur, z.plist);
    w.plist_cnt = carve<int>(cur, z.plist_cnt);
    w.pr = carve<d4>(cur, z.pr);
    w.tile_sums = carve<int2>(cur, z.tile_sums);
    w.max_chunks = z.max_chunks;
    w.list_cap = z.list_cap;
}

struct ProfRec {
    int kind;
    hipEvent_t a, b;
};

}  // namespace

// Per-evaluation buffers of ewald_energy_forces_noalloc(): one copy on every
// device the library runs on, held until the process ends.  Host code never
// passes this name to a kernel or a copy (on the host it is only a stand-in
// for the symbol); it uses the device address resolved once per device by
// scratch_address() below.
static __device__ __align__(256) unsigned char scratch[EWALD_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of this device's copy of `scratch`, resolved on the first
// call per device (with that device current) and kept; nullptr on failure.
void *scratch_address(int dev)
{
    if (dev < 0 || dev >= kMaxScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

struct ewald_plan_s {
    ewald_params prm{};
    hipStream_t stream = nullptr;
    // the reciprocal-space kernels run on a plan-owned stream, forked from and
    // joined back to the caller's stream, concurrently with the real-space ones
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_phase = nullptr;  // the phase tables are written (see phase_first)
    hipEvent_t ev_done = nullptr;  // recorded after each graph launch on the plan's stream
    bool last_graph = false;       // the previous evaluation was a graph launch
    int device = 0;
    bool mixed = false;
    int nc = 1, ncell = 1;
    int tile = 4;
    KLayout kl;
    Sizes sz{};
    void *base = nullptr;
    bool has_work = true;  // false: EWALD_FLAG_NO_WORKSPACE (tables only)
    void *scratch = nullptr;  // this device's static scratch (allocation-free evaluation)
    // plan-resident tables and status word
    int *status = nullptr;
    double *ck = nullptr;
    int *row_nx = nullptr, *row_ny = nullptr, *row_m = nullptr, *unit_g = nullptr, *unit_s = nullptr,
        *row_item = nullptr, *item_nx = nullptr, *item_ny = nullptr, *item_seg = nullptr;
    MTile *mtiles = nullptr;
    int *row_mbase = nullptr;
    int *unit_base = nullptr;
    int *sk_tile_of = nullptr;
    // the plan's own per-evaluation buffers (empty without a workspace)
    Work w;
    bool mfma_gather = false, mfma_sk = false;
    // graph replay of repeated evaluations (same n, buffers and kind)
    struct GraphKey {
        int64_t n = -1;
        const void *pos = nullptr, *q = nullptr, *energy = nullptr, *forces = nullptr, *dEdq = nullptr,
                   *gscale = nullptr;
        bool energy_only = false;
        bool operator==(const GraphKey &o) const
        {
            return n == o.n && pos == o.pos && q == o.q && energy == o.energy && forces == o.forces &&
                   dEdq == o.dEdq && gscale == o.gscale && energy_only == o.energy_only;
        }
    };
    struct GraphSlot {
        GraphKey key;
        hipGraphExec_t exec = nullptr;  // null until the key is seen a second time
        uint64_t used = 0;
    };
    static constexpr size_t kGraphSlots = 4;  // distinct keys kept (least recently used goes)
    bool graphs = true;          // false: plan flag, or a capture failed
    hipStream_t cap = nullptr;   // capture stream (the caller's may be the null stream)
    std::vector<GraphSlot> gslots;
    uint64_t gclock = 0;
    // profiling
    bool prof = false;
    std::vector<ProfRec> pending;
    std::vector<hipEvent_t> pool;
    double tot_ms[KC_COUNT] = {};
    int64_t launches[KC_COUNT] = {};
};

namespace {

class DeviceGuard {
  public:
    explicit DeviceGuard(int dev)
    {
        ok_ = hipGetDevice(&prev_) == hipSuccess;
        if (ok_ && prev_ != dev) ok_ = hipSetDevice(dev) == hipSuccess;
        restore_ = ok_ && prev_ != dev;
    }
    ~DeviceGuard()
    {
        if (restore_) (void)hipSetDevice(prev_);
    }
    bool ok() const { return ok_; }

  private:
    int prev_ = 0;
    bool ok_ = false, restore_ = false;
};

hipEvent_t take_event(ewald_plan_s *p)
{
    if (!p->pool.empty()) {
        hipEvent_t e = p->pool.back();
        p->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Runs one launcher on stream s, bracketed by events when profiling is on.
template <typename F>
hipError_t timed(ewald_plan_s *p, hipStream_t s, int kind, F &&launch)
{
    if (!p->prof) return launch();
    ProfRec r{kind, take_event(p), take_event(p)};
    if (r.a) (void)hipEventRecord(r.a, s);
    hipError_t e = launch();
    if (r.b) (void)hipEventRecord(r.b, s);
    if (r.a && r.b) p->pending.push_back(r);
    return e;
}

void drain_profile(ewald_plan_s *p)
{
    for (const ProfRec &r : p->pending) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            p->tot_ms[r.kind] += ms;
            p->launches[r.kind] += 1;
        }
        p->pool.push_back(r.a);
        p->pool.push_back(r.b);
    }
    p->pending.clear();
}

template <typename T>
hipError_t upload(T *dst, const std::vector<T> &src, hipStream_t s)
{
    if (src.empty()) return hipSuccess;
    return hipMemcpyAsync(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, s);
}

}  // namespace

extern "C" {

const char *ewald_status_string(ewald_status s)
{
    switch (s) {
    case EWALD_OK: return "ok";
    case EWALD_ERR_INVALID_ARG: return "invalid argument";
    case EWALD_ERR_CAPACITY: return "n exceeds the plan capacity n_max";
    case EWALD_ERR_OUT_OF_MEMORY: return "out of memory";
    case EWALD_ERR_DEVICE: return "HIP device or launch error";
    case EWALD_ERR_NONFINITE: return "non-finite position or charge";
    case EWALD_ERR_ADMISSION: return "plan workspace exceeds the server's free HBM budget";
    case EWALD_ERR_SCRATCH: return "buffers for this n exceed the static scratch (EWALD_SCRATCH_BYTES)";
    }
    return "unknown status";
}

ewald_status ewald_params_validate(const ewald_params *p)
{
    if (!p) return EWALD_ERR_INVALID_ARG;
    if (p->n_max < 1 || p->n_max > kPairMaxN) return EWALD_ERR_INVALID_ARG;
    if (!(std::isfinite(p->box_L) && p->box_L > 0.0)) return EWALD_ERR_INVALID_ARG;
    if (!(std::isfinite(p->alpha) && p->alpha > 0.0)) return EWALD_ERR_INVALID_ARG;
    if (!(std::isfinite(p->r_c) && p->r_c > 0.0 && p->r_c <= p->box_L)) return EWALD_ERR_INVALID_ARG;
    if (p->k_max < 1 || p->k_max > EWALD_K_MAX_LIMIT) return EWALD_ERR_INVALID_ARG;
    if (p->precision != EWALD_PRECISION_FP64 && p->precision != EWALD_PRECISION_MIXED) return EWALD_ERR_INVALID_ARG;
    if (p->device < 0 || (p->flags & ~(EWALD_FLAG_VALU_GATHER | EWALD_FLAG_VALU_SK | EWALD_FLAG_NO_GRAPH |
                                       EWALD_FLAG_NO_WORKSPACE | EWALD_FLAG_ONE_STREAM)) != 0)
        return EWALD_ERR_INVALID_ARG;
    return EWALD_OK;
}

int64_t ewald_kset_size(int32_t k_max)
{
    if (k_max < 1 || k_max > EWALD_K_MAX_LIMIT) return 0;
    int64_t c = 0;
    const int K2 = k_max * k_max;
    for (int nx = 0; nx <= k_max; ++nx)
        for (int ny = -k_max; ny <= k_max; ++ny)
            for (int nz = -k_max; nz <= k_max; ++nz) {
                const int m2 = nx * nx + ny * ny + nz * nz;
                if (m2 == 0 || m2 > K2) continue;
                if (nx > 0 || (ny > 0) || (ny == 0 && nz > 0)) ++c;
            }
    return c;
}

size_t ewald_plan_workspace_bytes(const ewald_params *p)
{
    if (ewald_params_validate(p) != EWALD_OK) return 0;
    KLayout kl;
    build_klayout(p->k_max, kl);
    Sizes z;
    compute_sizes(*p, kl, cells_per_axis(p->box_L, p->r_c), p->n_max, z);
    return z.total;
}

ewald_status ewald_plan(const ewald_params *params, ewald_plan_t *out)
{
    if (!out) return EWALD_ERR_INVALID_ARG;
    *out = nullptr;
    if (ewald_params_validate(params) != EWALD_OK) return EWALD_ERR_INVALID_ARG;
    ewald_plan_s *p = new (std::nothrow) ewald_plan_s();
    if (!p) return EWALD_ERR_OUT_OF_MEMORY;
    p->prm = *params;
    p->device = params->device;
    p->stream = reinterpret_cast<hipStream_t>(params->stream);
    p->mixed = params->precision == EWALD_PRECISION_MIXED;
    p->nc = cells_per_axis(params->box_L, params->r_c);
    p->ncell = p->nc * p->nc * p->nc;
    build_klayout(params->k_max, p->kl, !p->mixed);
    p->tile = sk_tile(params->k_max + 1);
    p->has_work = !(params->flags & EWALD_FLAG_NO_WORKSPACE);
    compute_sizes(*params, p->kl, p->nc, params->n_max, p->sz);

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || params->device >= ndev) {
        delete p;
        return ndev == 0 ? EWALD_ERR_DEVICE : EWALD_ERR_INVALID_ARG;
    }
    DeviceGuard dg(p->device);
    if (!dg.ok()) {
        delete p;
        return EWALD_ERR_DEVICE;
    }
    // set-up of the allocation-free evaluation on this device
    p->scratch = scratch_address(p->device);
    if (!p->has_work && !p->scratch) {
        delete p;
        return EWALD_ERR_DEVICE;
    }
    if (hipMalloc(&p->base, p->has_work ? p->sz.total : p->sz.tables) != hipSuccess) {
        (void)hipGetLastError();
        delete p;
        return EWALD_ERR_OUT_OF_MEMORY;
    }
    if (hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_phase, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        if (p->ev_phase) (void)hipEventDestroy(p->ev_phase);
        if (p->ev_join) (void)hipEventDestroy(p->ev_join);
        if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
        if (p->cap) (void)hipStreamDestroy(p->cap);
        if (p->aux) (void)hipStreamDestroy(p->aux);
        (void)hipFree(p->base);
        delete p;
        return EWALD_ERR_DEVICE;
    }
    char *cur = static_cast<char *>(p->base);
    const Sizes &z = p->sz;
    p->status = carve<int>(cur, z.status);
    p->ck = carve<double>(cur, z.ck);
    p->row_nx = carve<int>(cur, z.row_nx);
    p->row_ny = carve<int>(cur, z.row_ny);
    p->row_m = carve<int>(cur, z.row_m);
    p->unit_g = carve<int>(cur, z.unit_g);
    p->unit_s = carve<int>(cur, z.unit_s);
    p->row_item = carve<int>(cur, z.row_item);
    p->item_nx = carve<int>(cur, z.item_nx);
    p->item_ny = carve<int>(cur, z.item_ny);
    p->item_seg = carve<int>(cur, z.item_seg);
    p->mtiles = carve<MTile>(cur, z.mtiles);
    p->row_mbase = carve<int>(cur, z.row_mbase);
    p->unit_base = carve<int>(cur, z.unit_base);
    p->sk_tile_of = carve<int>(cur, z.sk_tile_of);
    if (p->has_work) carve_work(cur, z, p->w);
    p->graphs = !(params->flags & EWALD_FLAG_NO_GRAPH);
    p->mfma_sk = !(params->flags & EWALD_FLAG_VALU_SK) && p->kl.KP <= kSmMaxKP &&
                 sk_mfma_particles(p->kl.KP, !p->mixed) >= 8;
    // the matrix-core gather stages a block's z powers in at most 64 KB of LDS
    // (its x^n, y^n tables come on top: at most 86 KB at k_max 83 in FP64)
    p->mfma_gather = !(params->flags & EWALD_FLAG_VALU_GATHER) &&
                     gather_mfma_stage_bytes(p->kl.nap_max, gather_mfma_particles(params->n_max, !p->mixed),
                                             !p->mixed) <= 64 * 1024;

    // C_k by integer |n|^2 (computed once on the host in FP64)
    const int K = params->k_max;
    std::vector<double> ck((size_t)K * K + 1, 0.0);
    const double L = params->box_L, V = L * L * L, gk = 2.0 * kPi / L;
    for (int m2 = 1; m2 <= K * K; ++m2) {
        const double k2 = gk * gk * (double)m2;
        ck[m2] = 4.0 * kPi / (V * k2) * std::exp(-k2 / (4.0 * params->alpha));
    }
    hipError_t e = hipSuccess;
    const KLayout &kl = p->kl;
    hipStream_t s = p->stream;
    if (e == hipSuccess) e = upload(p->ck, ck, s);
    if (e == hipSuccess) e = upload(p->row_nx, kl.row_nx, s);
    if (e == hipSuccess) e = upload(p->row_ny, kl.row_ny, s);
    if (e == hipSuccess) e = upload(p->row_m, kl.row_m, s);
    if (e == hipSuccess) e = upload(p->unit_g, kl.unit_g, s);
    if (e == hipSuccess) e = upload(p->unit_s, kl.unit_s, s);
    if (e == hipSuccess) e = upload(p->row_item, kl.row_item, s);
    if (e == hipSuccess) e = upload(p->item_nx, kl.item_nx, s);
    if (e == hipSuccess) e = upload(p->item_ny, kl.item_ny, s);
    if (e == hipSuccess) e = upload(p->item_seg, kl.item_meta, s);
    if (e == hipSuccess) e = upload(p->mtiles, kl.mtiles, s);
    if (e == hipSuccess) e = upload(p->row_mbase, kl.row_mbase, s);
    if (e == hipSuccess) e = upload(p->unit_base, kl.unit_base, s);
    if (e == hipSuccess) e = upload(p->sk_tile_of, kl.sk_tile_of, s);
    if (e == hipSuccess) e = hipMemsetAsync(p->status, 0, z.status, s);
    if (p->has_work) {
        // padding entries of the tile coefficients are never written and stay zero
        if (e == hipSuccess) e = hipMemsetAsync(p->w.mcoef, 0, z.mcoef, s);
        // counters start at zero; afterwards every evaluation leaves them cleared
        if (e == hipSuccess) e = hipMemsetAsync(p->w.counts, 0, z.counts, s);
        if (e == hipSuccess) e = hipMemsetAsync(p->w.fill, 0, z.fill, s);
        if (e == hipSuccess) e = hipMemsetAsync(p->w.sk, 0, z.sk, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        (void)hipEventDestroy(p->ev_fork);
        (void)hipEventDestroy(p->ev_join);
        (void)hipEventDestroy(p->ev_phase);
        (void)hipEventDestroy(p->ev_done);
        (void)hipStreamDestroy(p->cap);
        (void)hipStreamDestroy(p->aux);
        (void)hipFree(p->base);
        delete p;
        return EWALD_ERR_DEVICE;
    }
    *out = p;
    return EWALD_OK;
}

ewald_status ewald_plan_set_stream(ewald_plan_t plan, void *stream)
{
    if (!plan) return EWALD_ERR_INVALID_ARG;
    plan->stream = reinterpret_cast<hipStream_t>(stream);
    return EWALD_OK;
}

}  // extern "C"

namespace {

// Position of a kernel class in the one-stream launch order (0: the workspace
// clear that precedes it).  A batch launches its systems' kernels class by
// class in this order.
int batch_rank(int kind)
{
    static const int rank[KC_COUNT] = {
        /* KC_BIN */ 5, /* KC_SCAN */ 6, /* KC_SCATTER */ 7, /* KC_CELLSORT */ 8,
        /* KC_PHASE */ 1, /* KC_SK */ 2, /* KC_SKREDUCE */ 3, /* KC_GATHER */ 4,
        /* KC_PAIRLIST */ 9, /* KC_PAIR */ 10, /* KC_FINAL_P */ 11, /* KC_FINAL_E */ 12};
    return rank[kind];
}

// Whether the real-space chain waits for the phase tables.  Started together,
// the real-space kernels (tens of thousands of small blocks) take the compute
// units from the phase kernel: at 10^6 ions it ran 3.6 ms beside them against
// 0.47 ms alone, on the reciprocal chain that sets the wall time.  Where the
// reciprocal work dominates, waiting costs the real-space chain little.  A pair
// costs about 31 (particle, k) terms (32^3: 114 us for 1.25e7 pairs against
// 157 us for 5.5e8 terms); the wait is taken when the reciprocal chain is
// estimated at three times the real-space one or more: |K+| ~ (2/3) pi K^3
// against 3 x 31 x (4/3) pi r_c^3 n / L^3 pairs per particle.  Measured: 10^6
// ions (ratio 3.9) 24.4 against 25.5 ms mixed, 33.0 against 33.9 FP64; 64^3
// (ratio 2.1) gained nothing mixed and lost 2 % in FP64, so it does not wait.
bool phase_first(const ewald_params &prm, int64_t n)
{
    const double L = prm.box_L, rc = prm.r_c, K = prm.k_max;
    const double pairs = 4.0 / 3.0 * kPi * rc * rc * rc * (double)n / (L * L * L);
    const double kvec = 2.0 / 3.0 * kPi * K * K * K;
    return kvec > 3.0 * 31.0 * pairs;
}

// The whole evaluation enqueued on stream s (the plan's stream, or its capture
// stream while a graph is recorded).  energy_only skips the force gather (the
// reciprocal energy comes from the structure factor alone); gscale, when
// given, turns the force / dE/dq outputs into the adjoint.
ewald_status launch_path(ewald_plan_t p, const Work &w, hipStream_t s, bool one_stream, int64_t n,
                         const double *pos, const double *q, double *energy, double *forces, double *dEdq,
                         const double *gscale, bool energy_only, bool allow_prof = true)
{
    const KLayout &kl = p->kl;
    const double L = p->prm.box_L;

    CellArgs ca{n, L, p->nc, p->ncell};
    RecipArgs ra{n, L, kl.K, kl.KP, kl.n_rows, kl.n_units, kl.n_items, kl.n_units * kQ * kLanes};
    PairArgs pa{n, L, p->nc, p->ncell, p->prm.r_c * p->prm.r_c, p->prm.alpha};
    int n_chunks = sk_chunks(n, kl.n_units, p->tile);
    if (p->mfma_sk) {
        // particle chunks of the matrix-core structure factor: fill the chip, at
        // most the partial-sum capacity, at least one staged tile per chunk
        int64_t c = sk_mfma_target_blocks() / sk_mfma_row_blocks(kl.n_rows);
        c = std::min<int64_t>(c, w.max_chunks);
        const int P = sk_mfma_particles(kl.KP, !p->mixed);
        c = std::min<int64_t>(c, (n + P - 1) / P);
        n_chunks = (int)std::max<int64_t>(c, 1);
    }
    const int chunk_len = (int)((n + n_chunks - 1) / n_chunks);
    const int n_split = p->mfma_gather ? gather_mfma_split(n, kl, !p->mixed) : gather_split(n);
    SplitTable st{};
    if (p->mfma_gather)
        mfma_split_table(kl, n_split, st);
    else
        for (int k = 0; k <= n_split; ++k) st.lo[k] = (int)((int64_t)kl.n_items * k / n_split);
    FinalArgs fa{n, L, p->prm.alpha, energy_only ? 0 : n_split, ceil_div((int64_t)ra.n_slots, 256 / kRedSlotLanes),
                 gscale};
    const int nqb = bin_blocks(n);

    hipError_t e = hipSuccess;
    auto run = [&](hipStream_t st, int kind, auto &&fn) {
        if (e != hipSuccess) return;
        if (t_batch) {
            t_batch->kind = batch_rank(kind);
            t_batch->occ = 0;
        }
        e = allow_prof ? timed(p, st, kind, fn) : fn();
    };
    // Reciprocal space on the plan's own stream, from the caller's positions and
    // charges: it needs nothing from the cell list, so it runs beside the real
    // space.  Phase tables and the structure factor are FP64 in both precisions
    // (FP32 phase rounding leaves ~1e-5 relative error in S_k of near-lattice
    // systems at small k); the mixed path rounds phases and coefficients to
    // FP32 in the gather and evaluates the pair functions in FP32.
    // one_stream: everything in order on s (no fork, no events)
    one_stream = one_stream || (p->prm.flags & EWALD_FLAG_ONE_STREAM) != 0;
    hipStream_t ax = one_stream ? s : p->aux;
    if (!one_stream) {
        if (e == hipSuccess) e = hipEventRecord(p->ev_fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(ax, p->ev_fork, 0);
    }
    {
        auto *tx = static_cast<c64 *>(w.tx), *ty = static_cast<c64 *>(w.ty), *tz = static_cast<c64 *>(w.tz);
        run(ax, KC_PHASE, [&] { return launch_phase<double>(ax, ra, pos, q, w.pr, tx, ty, tz); });
        if (!one_stream && e == hipSuccess && phase_first(p->prm, n)) {
            e = hipEventRecord(p->ev_phase, ax);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, p->ev_phase, 0);
        }
        run(ax, KC_SK, [&] {
            if (p->mfma_sk)
                return launch_sk_mfma(ax, ra, n_chunks, chunk_len, tx, ty, tz, p->row_nx, p->row_ny,
                                      p->row_m, p->unit_base, p->sk_tile_of, w.part, !p->mixed);
            return launch_sk(ax, ra, n_chunks, chunk_len, tx, ty, tz, p->unit_g, p->unit_s, p->row_nx, p->row_ny,
                             w.part);
        });
        if (p->mixed) {
            float *rec = p->mfma_gather ? nullptr : static_cast<float *>(w.rec);
            float *mc = p->mfma_gather ? static_cast<float *>(w.mcoef) : nullptr;
            run(ax, KC_SKREDUCE, [&] {
                return launch_sk_reduce<float>(ax, ra, n_chunks, w.part, p->unit_g, p->unit_s, p->row_nx,
                                               p->row_ny, p->row_m, p->row_item, p->ck, w.sk, rec, mc,
                                               p->row_mbase, w.erec);
            });
            if (!energy_only) run(ax, KC_GATHER, [&] {
                if (p->mfma_gather)
                    return launch_gather_mfma<float>(ax, ra, n_split, st, kl.nap_max, w.pr, tz, p->mtiles, mc,
                                                     w.gpart);
                return launch_gather<float>(ax, ra, n_split, st, w.pr, tz, p->item_seg, rec, w.gpart);
            });
        } else {
            double *rec = p->mfma_gather ? nullptr : static_cast<double *>(w.rec);
            double *mc = p->mfma_gather ? static_cast<double *>(w.mcoef) : nullptr;
            run(ax, KC_SKREDUCE, [&] {
                return launch_sk_reduce<double>(ax, ra, n_chunks, w.part, p->unit_g, p->unit_s, p->row_nx,
                                                p->row_ny, p->row_m, p->row_item, p->ck, w.sk, rec, mc,
                                                p->row_mbase, w.erec);
            });
            if (!energy_only) run(ax, KC_GATHER, [&] {
                if (p->mfma_gather)
                    return launch_gather_mfma<double>(ax, ra, n_split, st, kl.nap_max, w.pr, tz, p->mtiles, mc,
                                                      w.gpart);
                return launch_gather<double>(ax, ra, n_split, st, w.pr, tz, p->item_seg, rec, w.gpart);
            });
        }
    }
    if (!one_stream && e == hipSuccess) e = hipEventRecord(p->ev_join, ax);

    // Real space on the caller's stream.
    if (cells_small(ca)) {  // one workgroup, same results
        run(s, KC_BIN, [&] {
            return launch_cells_small(s, ca, pos, q, w.cell_start, w.pitem_cell, w.pitem_off, w.n_pitems, w.scalars,
                                      w.perm, w.pq, p->status);
        });
    } else {
        run(s, KC_BIN, [&] { return launch_bin(s, ca, pos, q, w.cell_of, w.counts, w.qpart, p->status); });
        run(s, KC_SCAN, [&] {
            return launch_scan(s, ca, w.counts, w.fill, w.cell_start, w.qpart, nqb, w.scalars, w.tile_sums,
                               w.pitem_cell, w.pitem_off, w.n_pitems);
        });
        run(s, KC_SCATTER, [&] { return launch_scatter(s, ca, w.cell_of, w.cell_start, w.fill, w.tmp_idx); });
        run(s, KC_CELLSORT,
            [&] { return launch_cellsort(s, ca, w.cell_start, w.tmp_idx, pos, q, w.perm, w.pq); });
    }
    const int max_pitems = p->ncell + ceil_div(n, kPairHome);
    run(s, KC_PAIRLIST, [&] {
        return launch_pair_list(s, pa, max_pitems, w.n_pitems, w.pitem_cell, w.pitem_off, w.cell_start, w.pq,
                                w.plist, w.plist_cnt, w.list_cap);
    });
    run(s, KC_PAIR, [&] {
        return launch_pair(s, pa, p->mixed, w.cell_start, w.pq, w.plist, w.plist_cnt, w.list_cap, w.freal);
    });

    // Join, then the totals.
    if (!one_stream && e == hipSuccess) e = hipStreamWaitEvent(s, p->ev_join, 0);
    if (finalize_small(n)) {  // one workgroup, same sums
        run(s, KC_FINAL_P, [&] {
            return launch_finalize_small(s, fa, w.pq, w.perm, w.freal, w.gpart, w.scalars, forces, dEdq, w.erec,
                                         p->status, energy);
        });
    } else {
        run(s, KC_FINAL_P, [&] {
            return launch_finalize_particles(s, fa, w.pq, w.perm, w.freal, w.gpart, w.scalars, forces, dEdq,
                                             w.epart);
        });
        run(s, KC_FINAL_E, [&] {
            return launch_finalize_energy(s, fa, w.epart, ceil_div(n, 256), w.erec, w.scalars, p->status, energy);
        });
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return EWALD_ERR_DEVICE;
    }
    return EWALD_OK;
}

// Kernel-by-kernel launch, or graph replay when the evaluation repeats an
// earlier one's key (one of the last kGraphSlots distinct keys): the second
// evaluation with a key records the launch sequence on the capture stream (the
// reciprocal stream joins the capture through the fork event) and every later
// one on an idle stream launches that graph.
ewald_status run_path(ewald_plan_t p, int64_t n, const double *pos, const double *q, double *energy, double *forces,
                      double *dEdq, const double *gscale, bool energy_only)
{
    if (!p->has_work) return EWALD_ERR_INVALID_ARG;
    if (n > p->prm.n_max) return EWALD_ERR_CAPACITY;
    DeviceGuard dg(p->device);
    if (!dg.ok()) return EWALD_ERR_DEVICE;
    if (p->prof || !p->graphs) return launch_path(p, p->w, p->stream, false, n, pos, q, energy, forces, dEdq, gscale, energy_only);
    ewald_plan_s::GraphKey key;
    key.n = n;
    key.pos = pos;
    key.q = q;
    key.energy = energy;
    key.forces = forces;
    key.dEdq = dEdq;
    key.gscale = gscale;
    key.energy_only = energy_only;
    // A graph launch is followed by the completion event; a kernel-by-kernel
    // evaluation already records the join event at the end of its reciprocal
    // chain, which serves as its (nearly complete) marker.  No marker is added
    // to the eager path, so back-to-back evaluations keep their packet stream.
    auto eager = [&]() {
        p->last_graph = false;
        return launch_path(p, p->w, p->stream, false, n, pos, q, energy, forces, dEdq, gscale, energy_only);
    };
    auto graph = [&](hipGraphExec_t x) {
        p->last_graph = true;
        if (hipGraphLaunch(x, p->stream) != hipSuccess) return EWALD_ERR_DEVICE;
        return hipEventRecord(p->ev_done, p->stream) == hipSuccess ? EWALD_OK : EWALD_ERR_DEVICE;
    };
    ewald_plan_s::GraphSlot *slot = nullptr;
    for (auto &sl : p->gslots)
        if (sl.key == key) slot = &sl;
    if (!slot) {
        // first sight of this key: remember it (evicting the least recently used)
        if (p->gslots.size() < ewald_plan_s::kGraphSlots) {
            p->gslots.emplace_back();
            slot = &p->gslots.back();
        } else {
            slot = &p->gslots[0];
            for (auto &sl : p->gslots)
                if (sl.used < slot->used) slot = &sl;
            if (slot->exec) (void)hipGraphExecDestroy(slot->exec);
            slot->exec = nullptr;
        }
        slot->key = key;
        slot->used = ++p->gclock;
        return eager();
    }
    slot->used = ++p->gclock;
    if (slot->exec) {
        // A graph launch saves host launch time, which is what a call on an idle
        // stream waits for; with work already queued the kernels run faster
        // launched one by one (measured at 32^3: 0.235 against 0.242 ms back to
        // back, 0.28 against 0.26 ms per synchronised call), so the graph is
        // used only on an idle stream.
        // Idle: the previous evaluation's marker has fired.
        const hipError_t busy = hipEventQuery(p->last_graph ? p->ev_done : p->ev_join);
        if (busy == hipErrorNotReady) {
            (void)hipGetLastError();
            return eager();
        }
        return graph(slot->exec);
    }
    // second evaluation with this key: record it
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    ewald_status st = EWALD_ERR_DEVICE;
    if (hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        st = launch_path(p, p->w, p->cap, false, n, pos, q, energy, forces, dEdq, gscale, energy_only);
        const hipError_t ec = hipStreamEndCapture(p->cap, &g);
        if (ec != hipSuccess || !g) st = EWALD_ERR_DEVICE;
        if (st == EWALD_OK && hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
            x = nullptr;
            st = EWALD_ERR_DEVICE;
        }
        if (g) (void)hipGraphDestroy(g);
    }
    if (st != EWALD_OK || !x) {
        // no graphs for this plan: launch kernel by kernel from now on
        (void)hipGetLastError();
        if (x) (void)hipGraphExecDestroy(x);
        p->graphs = false;
        return eager();
    }
    slot->exec = x;
    return graph(x);
}

}  // namespace

extern "C" {

ewald_status ewald_energy_forces(ewald_plan_t p, int64_t n, const double *pos, const double *q, double *energy,
                                 double *forces, double *dEdq)
{
    if (!p || !pos || !q || !energy || n < 1) return EWALD_ERR_INVALID_ARG;
    if (n > p->prm.n_max) return EWALD_ERR_CAPACITY;
    return run_path(p, n, pos, q, energy, forces, dEdq, nullptr, false);
}

size_t ewald_eval_workspace_bytes(ewald_plan_t p, int64_t n)
{
    if (!p || n < 1 || n > p->prm.n_max) return 0;
    Sizes z;
    compute_sizes(p->prm, p->kl, p->nc, n, z);
    return z.work;
}

}  // extern "C"

namespace {

// One evaluation whose per-evaluation buffers are carved from `base` (sized for
// n by compute_sizes): the counters and padding that must start at zero are
// cleared first, then the kernels are launched one by one.
ewald_status run_in_buffers(ewald_plan_t p, int64_t n, const double *pos, const double *q, double *energy,
                            double *forces, double *dEdq, void *base, const Sizes &z)
{
    DeviceGuard dg(p->device);
    if (!dg.ok()) return EWALD_ERR_DEVICE;
    Work w;
    carve_work(static_cast<char *>(base), z, w);
    if (launch_zero(p->stream, base, zeroed_bytes(z)) != hipSuccess) {
        (void)hipGetLastError();
        return EWALD_ERR_DEVICE;
    }
    p->last_graph = false;  // this call's join event marks its completion
    return launch_path(p, w, p->stream, false, n, pos, q, energy, forces, dEdq, nullptr, false, false);
}

}  // namespace

extern "C" {

ewald_status ewald_energy_forces_ws(ewald_plan_t p, int64_t n, const double *pos, const double *q, double *energy,
                                    double *forces, double *dEdq, void *workspace, size_t workspace_bytes)
{
    if (!p || !pos || !q || !energy || n < 1 || !workspace || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return EWALD_ERR_INVALID_ARG;
    if (n > p->prm.n_max) return EWALD_ERR_CAPACITY;
    Sizes z;
    compute_sizes(p->prm, p->kl, p->nc, n, z);
    if (z.work > workspace_bytes) return EWALD_ERR_CAPACITY;
    return run_in_buffers(p, n, pos, q, energy, forces, dEdq, workspace, z);
}

ewald_status ewald_energy_forces_noalloc(ewald_plan_t p, int64_t n, const double *pos, const double *q,
                                         double *energy, double *forces, double *dEdq)
{
    if (!p || !pos || !q || !energy || n < 1) return EWALD_ERR_INVALID_ARG;
    if (n > p->prm.n_max) return EWALD_ERR_CAPACITY;
    Sizes z;
    compute_sizes(p->prm, p->kl, p->nc, n, z);
    if (z.work > EWALD_SCRATCH_BYTES) return EWALD_ERR_SCRATCH;
    if (!p->scratch) return EWALD_ERR_DEVICE;
    // the array keeps whatever the last call on this device left in it
    return run_in_buffers(p, n, pos, q, energy, forces, dEdq, p->scratch, z);
}

ewald_status ewald_energy_forces_batch(int32_t count, const ewald_plan_t *plans, const int64_t *n,
                                       const double *const *pos, const double *const *q, double *const *energy,
                                       double *const *forces, double *const *dEdq, void *const *workspace,
                                       const size_t *workspace_bytes, void *stream)
{
    if (count < 1 || count > EWALD_BATCH_MAX || !plans || !n || !pos || !q || !energy) return EWALD_ERR_INVALID_ARG;
    if (!plans[0]) return EWALD_ERR_INVALID_ARG;
    const int dev = plans[0]->device;
    std::vector<Sizes> zs((size_t)count);
    for (int i = 0; i < count; ++i) {
        ewald_plan_t p = plans[i];
        if (!p || p->device != dev || !pos[i] || !q[i] || !energy[i] || n[i] < 1) return EWALD_ERR_INVALID_ARG;
        if (n[i] > p->prm.n_max) return EWALD_ERR_CAPACITY;
        void *ws = workspace ? workspace[i] : nullptr;
        if (ws) {
            if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return EWALD_ERR_INVALID_ARG;
            compute_sizes(p->prm, p->kl, p->nc, n[i], zs[i]);
            if (!workspace_bytes || zs[i].work > workspace_bytes[i]) return EWALD_ERR_CAPACITY;
        } else {
            // the plan's own buffers serve one system of the batch at most
            if (!p->has_work) return EWALD_ERR_INVALID_ARG;
            for (int j = 0; j < i; ++j)
                if (plans[j] == p && !(workspace && workspace[j])) return EWALD_ERR_INVALID_ARG;
        }
    }
    DeviceGuard dg(dev);
    if (!dg.ok()) return EWALD_ERR_DEVICE;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    // 1. every system's launch sequence, recorded instead of launched
    BatchRecorder rec;
    {
        struct Install {
            explicit Install(BatchRecorder *r) { t_batch = r; }
            ~Install() { t_batch = nullptr; }
        } install(&rec);
        for (int i = 0; i < count; ++i) {
            ewald_plan_t p = plans[i];
            rec.sys = i;
            Work w = p->w;
            void *ws = workspace ? workspace[i] : nullptr;
            if (ws) {
                carve_work(static_cast<char *>(ws), zs[i], w);
                rec.kind = 0;
                rec.occ = 0;
                (void)launch_zero(s, ws, zeroed_bytes(zs[i]));
            }
            p->last_graph = false;
            const ewald_status st = launch_path(p, w, s, true, n[i], pos[i], q[i], energy[i],
                                                forces ? forces[i] : nullptr, dEdq ? dEdq[i] : nullptr, nullptr,
                                                false, false);
            if (st != EWALD_OK) return st;
        }
    }
    // 2. one launch per (kernel class, occurrence, kernel instance, block
    // size), in the launch order of a single evaluation: each system's
    // launches keep their order, and the launches of one class run together
    const std::vector<LaunchRecord> &r = rec.recs;
    for (size_t k = 1; k < r.size(); ++k)
        if (r[k].sys == r[k - 1].sys &&
            (r[k].kind < r[k - 1].kind || (r[k].kind == r[k - 1].kind && r[k].occ <= r[k - 1].occ)))
            return EWALD_ERR_DEVICE;  // not in launch order (not expected)
    std::vector<int> order(r.size());
    for (size_t k = 0; k < r.size(); ++k) order[k] = (int)k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return r[a].kind != r[b].kind ? r[a].kind < r[b].kind : r[a].occ < r[b].occ;
    });
    std::vector<unsigned char> pack;
    hipError_t e = hipSuccess;
    // As in a single evaluation, the reciprocal-space classes run on a second
    // stream (plans[0]'s), forked from and joined back to `stream`, beside the
    // real-space ones, unless plans[0] keeps everything on one stream.
    ewald_plan_t p0 = plans[0];
    const bool two = (p0->prm.flags & EWALD_FLAG_ONE_STREAM) == 0;
    bool forked = false, joined = false;
    auto fork = [&] {
        if (!two || forked || e != hipSuccess) return;
        e = hipEventRecord(p0->ev_fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(p0->aux, p0->ev_fork, 0);
        forked = true;
    };
    auto join = [&] {
        if (!forked || joined || e != hipSuccess) return;
        e = hipEventRecord(p0->ev_join, p0->aux);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, p0->ev_join, 0);
        joined = true;
    };
    for (size_t lo = 0; lo < order.size() && e == hipSuccess;) {
        size_t hi = lo;
        while (hi < order.size() && r[order[hi]].kind == r[order[lo]].kind && r[order[hi]].occ == r[order[lo]].occ)
            ++hi;
        const int kind = r[order[lo]].kind;
        if (kind >= batch_rank(KC_PHASE)) fork();
        if (kind >= batch_rank(KC_FINAL_P)) join();
        const bool recip = kind >= batch_rank(KC_PHASE) && kind < batch_rank(KC_BIN);
        const hipStream_t ls = forked && !joined && recip ? p0->aux : s;
        std::vector<bool> done(hi - lo, false);
        for (size_t g = lo; g < hi && e == hipSuccess; ++g) {
            if (done[g - lo]) continue;
            const LaunchRecord &head = r[order[g]];
            std::vector<int> members;
            for (size_t m = g; m < hi; ++m)
                if (!done[m - lo] && r[order[m]].many == head.many && r[order[m]].threads == head.threads) {
                    members.push_back(order[m]);
                    done[m - lo] = true;
                }
            // at most cap systems per launch
            for (size_t c0 = 0; c0 < members.size() && e == hipSuccess; c0 += (size_t)head.cap) {
                const size_t c1 = std::min(members.size(), c0 + (size_t)head.cap);
                pack.assign(head.pack_size, 0);
                BatchSpan *span = reinterpret_cast<BatchSpan *>(pack.data() + head.span_off);
                int64_t blocks = 0;
                size_t smem = 0;
                for (size_t m = c0; m < c1; ++m) {
                    const LaunchRecord &x = r[members[m]];
                    std::memcpy(pack.data() + (m - c0) * head.args_size, rec.args.data() + x.args_off, head.args_size);
                    span[m - c0].first = (int)blocks;
                    span[m - c0].gx = (int)x.grid.x;
                    blocks += (int64_t)x.grid.x * x.grid.y * x.grid.z;
                    smem = std::max(smem, x.smem);
                }
                span[c1 - c0].first = (int)blocks;
                const int nsys = (int)(c1 - c0);
                std::memcpy(pack.data() + head.nsys_off, &nsys, sizeof(int));
                if (blocks == 0) continue;
                if (blocks > INT32_MAX) {
                    e = hipErrorInvalidConfiguration;
                    break;
                }
                void *argv[] = {pack.data()};
                e = hipLaunchKernel(head.many, dim3((unsigned)blocks), dim3((unsigned)head.threads), argv, smem, ls);
            }
        }
        lo = hi;
    }
    join();
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return EWALD_ERR_DEVICE;
    }
    return EWALD_OK;
}

ewald_status ewald_energy(ewald_plan_t p, int64_t n, const double *pos, const double *q, double *energy)
{
    if (!p || !pos || !q || !energy || n < 1) return EWALD_ERR_INVALID_ARG;
    if (n > p->prm.n_max) return EWALD_ERR_CAPACITY;
    return run_path(p, n, pos, q, energy, nullptr, nullptr, nullptr, true);
}

ewald_status ewald_energy_backward(ewald_plan_t p, int64_t n, const double *pos, const double *q,
                                   const double *grad_energy, double *energy, double *grad_pos, double *grad_q)
{
    if (!p || !pos || !q || !grad_energy || !energy || n < 1) return EWALD_ERR_INVALID_ARG;
    if (n > p->prm.n_max) return EWALD_ERR_CAPACITY;
    return run_path(p, n, pos, q, energy, grad_pos, grad_q, grad_energy, false);
}

ewald_status ewald_plan_status(ewald_plan_t p)
{
    if (!p) return EWALD_ERR_INVALID_ARG;
    DeviceGuard dg(p->device);
    if (!dg.ok()) return EWALD_ERR_DEVICE;
    int st[2] = {0, 0};
    if (hipStreamSynchronize(p->stream) != hipSuccess) return EWALD_ERR_DEVICE;
    if (hipMemcpy(st, p->status, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess) return EWALD_ERR_DEVICE;
    if (st[1] || st[0]) {
        const int zero[2] = {0, 0};
        if (hipMemcpy(p->status, zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess) return EWALD_ERR_DEVICE;
        return EWALD_ERR_NONFINITE;
    }
    return EWALD_OK;
}

void ewald_release(ewald_plan_t p)
{
    if (!p) return;
    {
        DeviceGuard dg(p->device);
        (void)hipStreamSynchronize(p->stream);
        (void)hipStreamSynchronize(p->aux);
        for (const auto &slot : p->gslots)
            if (slot.exec) (void)hipGraphExecDestroy(slot.exec);
        (void)hipEventDestroy(p->ev_fork);
        (void)hipEventDestroy(p->ev_join);
        (void)hipEventDestroy(p->ev_phase);
        (void)hipEventDestroy(p->ev_done);
        (void)hipStreamDestroy(p->cap);
        (void)hipStreamDestroy(p->aux);
        for (const ProfRec &r : p->pending) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (hipEvent_t ev : p->pool) (void)hipEventDestroy(ev);
        if (p->base) (void)hipFree(p->base);
    }
    delete p;
}

int64_t ewald_plan_kcount(ewald_plan_t p) { return p ? p->kl.kcount : 0; }

// k vectors in slot order: for each slot (unit, a-offset, lane) the +a vector,
// then the -a vector when it belongs to K+.
static void slot_kvecs(const KLayout &kl, std::vector<int> &kv, std::vector<int64_t> &src)
{
    const int n_slots = kl.n_units * kQ * kLanes;
    kv.clear();
    src.clear();
    for (int slot = 0; slot < n_slots; ++slot) {
        const int lane = slot % kLanes, uq = slot / kLanes, k = uq % kQ, u = uq / kQ;
        const int r = kl.unit_g[u] * kLanes + lane;
        if (r >= kl.n_rows) continue;
        const int a = kl.unit_s[u] * kQ + k;
        if (a > kl.row_m[r]) continue;
        const int nx = kl.row_nx[r], ny = kl.row_ny[r];
        const bool axis = nx == 0 && ny == 0;
        if (!(axis && a == 0)) {
            kv.insert(kv.end(), {nx, ny, a});
            src.push_back(2 * (int64_t)slot);
        }
        if (a > 0 && !axis) {
            kv.insert(kv.end(), {nx, ny, -a});
            src.push_back(2 * (int64_t)slot + 1);
        }
    }
}

ewald_status ewald_debug_kset(ewald_plan_t p, int32_t *n_xyz)
{
    if (!p || !n_xyz) return EWALD_ERR_INVALID_ARG;
    std::vector<int> kv;
    std::vector<int64_t> src;
    slot_kvecs(p->kl, kv, src);
    for (size_t i = 0; i < kv.size(); ++i) n_xyz[i] = kv[i];
    return EWALD_OK;
}

ewald_status ewald_debug_copy_sk(ewald_plan_t p, double *re, double *im)
{
    if (!p || !re || !im || !p->has_work) return EWALD_ERR_INVALID_ARG;
    DeviceGuard dg(p->device);
    if (!dg.ok()) return EWALD_ERR_DEVICE;
    const int n_slots = p->kl.n_units * kQ * kLanes;
    std::vector<d4> h((size_t)n_slots);
    if (hipStreamSynchronize(p->stream) != hipSuccess) return EWALD_ERR_DEVICE;
    if (hipMemcpy(h.data(), p->w.sk, sizeof(d4) * n_slots, hipMemcpyDeviceToHost) != hipSuccess)
        return EWALD_ERR_DEVICE;
    std::vector<int> kv;
    std::vector<int64_t> src;
    slot_kvecs(p->kl, kv, src);
    for (size_t i = 0; i < src.size(); ++i) {
        const d4 &v = h[src[i] / 2];
        re[i] = (src[i] & 1) ? v.c : v.a;
        im[i] = (src[i] & 1) ? v.d : v.b;
    }
    return EWALD_OK;
}

ewald_status ewald_debug_stats_read(ewald_plan_t p, int64_t n, ewald_debug_stats *out)
{
    if (!p || !out || n < 1 || n > p->prm.n_max || !p->has_work) return EWALD_ERR_INVALID_ARG;
    DeviceGuard dg(p->device);
    if (!dg.ok()) return EWALD_ERR_DEVICE;
    std::vector<int> cs((size_t)p->ncell + 1), cnt((size_t)n);
    if (hipStreamSynchronize(p->stream) != hipSuccess) return EWALD_ERR_DEVICE;
    if (hipMemcpy(cs.data(), p->w.cell_start, sizeof(int) * cs.size(), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(cnt.data(), p->w.plist_cnt, sizeof(int) * cnt.size(), hipMemcpyDeviceToHost) != hipSuccess)
        return EWALD_ERR_DEVICE;
    std::memset(out, 0, sizeof(*out));
    for (int c = 0; c < p->ncell; ++c) out->max_cell_count = std::max<int64_t>(out->max_cell_count, cs[c + 1] - cs[c]);
    for (int v : cnt) {
        out->direct_particles += v < 0;
        out->listed_pairs += v > 0 ? v : 0;
    }
    out->cells_per_axis = p->nc;
    out->list_capacity = p->sz.list_cap;
    out->sk_matrix_cores = p->mfma_sk;
    out->gather_matrix_cores = p->mfma_gather;
    out->phase_rows = phase_rows<double>(p->kl.KP);
    // Matrix-core work per launch, from the launch shapes launch_path uses.
    const KLayout &kl = p->kl;
    if (p->mfma_sk) {
        // every staged sub-chunk of P particles: P / 4 quads x 2 MFMAs (Re U, Im U)
        // per pair of a of each tile
        int64_t naps = 0;
        for (int t : kl.sk_tile_of)
            if (t >= 0) naps += (kl.row_m[(size_t)t * kSmTileRows] + 2) / 2;
        const int P = sk_mfma_particles(kl.KP, !p->mixed);
        int64_t c = sk_mfma_target_blocks() / sk_mfma_row_blocks(kl.n_rows);
        c = std::min<int64_t>(c, p->w.max_chunks);
        c = std::min<int64_t>(c, (n + P - 1) / P);
        const int64_t n_chunks = std::max<int64_t>(c, 1), chunk_len = (n + n_chunks - 1) / n_chunks;
        int64_t subchunks = 0;
        for (int64_t k = 0; k < n_chunks; ++k) {
            const int64_t len = std::max<int64_t>(0, std::min<int64_t>(chunk_len, n - k * chunk_len));
            subchunks += (len + P - 1) / P;
        }
        out->sk_mfma_flops = subchunks * (P / 4) * 2 * naps * 512;
    }
    if (p->mfma_gather) {
        // every block of np particles: 4 quantities x np / 16 sub-tiles per pair of a of every tile
        int64_t naps = 0;
        for (const MTile &t : kl.mtiles) naps += t.nap;
        const int np = gather_mfma_particles(n, !p->mixed);
        const int64_t blocks = (n + np - 1) / np;
        out->gather_mfma_flops = blocks * 4 * (np / 16) * naps * 2048;
    }
    return EWALD_OK;
}

ewald_status ewald_profile_enable(ewald_plan_t p, int32_t enable)
{
    if (!p) return EWALD_ERR_INVALID_ARG;
    p->prof = enable != 0;
    return EWALD_OK;
}

int32_t ewald_profile_read(ewald_plan_t p, const char **names, double *total_ms, int64_t *launches,
                           int32_t max_entries)
{
    if (!p) return 0;
    {
        DeviceGuard dg(p->device);
        drain_profile(p);
    }
    const int n = std::min<int>(KC_COUNT, max_entries);
    for (int k = 0; k < n; ++k) {
        if (names) names[k] = kKernelClassNames[k];
        if (total_ms) total_ms[k] = p->tot_ms[k];
        if (launches) launches[k] = p->launches[k];
    }
    return KC_COUNT;
}

ewald_status ewald_profile_reset(ewald_plan_t p)
{
    if (!p) return EWALD_ERR_INVALID_ARG;
    {
        DeviceGuard dg(p->device);
        drain_profile(p);
    }
    for (int k = 0; k < KC_COUNT; ++k) {
        p->tot_ms[k] = 0.0;
        p->launches[k] = 0;
    }
    return EWALD_OK;
}

}  // extern "C"
