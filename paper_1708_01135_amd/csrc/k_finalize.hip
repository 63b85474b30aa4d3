// Totals and output (section 3.2.2 for the self term):
//   F_i      = F_real,i + q_i (2 pi / L) sum_splits g_i            (caller order;
//              the real-space sums are in cell order, the reciprocal ones in caller order)
//   with an upstream gradient g (device scalar) the outputs become the adjoint
//   dL/dr_i = -g F_i and dL/dq_i = g dE/dq_i.
//   dE/dq_i  = phi_real,i + phi_recip,i - 2 sqrt(alpha/pi) q_i - pi Q / (V alpha)
//   E_real   = 1/2 sum_i q_i phi_real,i
//   E_self   = -sqrt(alpha/pi) sum q_i^2,   E_bg = -pi Q^2 / (2 V alpha)
// All sums run in a fixed order (per-block trees, then one ordered pass); a
// small system takes both passes in one workgroup with the same sums.
#include "ewald_internal.h"

namespace ewk {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

// Outputs of cell-ordered particle s; returns its share 1/2 q_i phi_real,i of
// the real-space energy (0 past n).
__device__ inline double final_particle(int64_t s, int64_t n, double L, double alpha, int n_split,
                                        const d4 *__restrict__ pq, const int *__restrict__ perm,
                                        const d4 *__restrict__ freal, const d4 *__restrict__ gpart,
                                        const double *__restrict__ scalars, const double *__restrict__ gscale,
                                        double *__restrict__ forces, double *__restrict__ dEdq)
{
    if (s >= n) return 0.0;
    const d4 fr = freal[s];
    const int64_t i = perm[s];
    double g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
    for (int sp = 0; sp < n_split; ++sp) {
        const d4 g = gpart[(size_t)sp * n + i];
        g0 += g.a;
        g1 += g.b;
        g2 += g.c;
        g3 += g.d;
    }
    const double q = pq[s].d;
    const double kf = q * (2.0 * kPi / L);
    const double gs = gscale ? *gscale : 1.0;
    const double fs = gscale ? -gs : 1.0;
    if (forces) {
        forces[3 * i] = fs * (fr.b + kf * g1);
        forces[3 * i + 1] = fs * (fr.c + kf * g2);
        forces[3 * i + 2] = fs * (fr.d + kf * g3);
    }
    if (dEdq) {
        const double V = L * L * L;
        dEdq[i] = gs * (fr.a + g0 - 2.0 * sqrt(alpha / kPi) * q - kPi * scalars[0] / (V * alpha));
    }
    return 0.5 * q * fr.a;
}

// Tree over 256 values of one block (thread t holds sh[t] on entry).
__device__ inline double block_tree256(double *sh)
{
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    return sh[0];
}

__device__ __forceinline__ void final_p_body(int bx, int by, int64_t n, double L, double alpha, int n_split,
                                             const d4 *__restrict__ pq, const int *__restrict__ perm,
                                             const d4 *__restrict__ freal, const d4 *__restrict__ gpart,
                                             const double *__restrict__ scalars, const double *__restrict__ gscale,
                                             double *__restrict__ forces, double *__restrict__ dEdq,
                                             double *__restrict__ epart)
{
    __shared__ double s_e[256];
    const int64_t s = (int64_t)bx * 256 + threadIdx.x;
    s_e[threadIdx.x] = final_particle(s, n, L, alpha, n_split, pq, perm, freal, gpart, scalars, gscale, forces, dEdq);
    const double e = block_tree256(s_e);
    if (threadIdx.x == 0) epart[bx] = e;
}

struct KFinalP {
    static constexpr int kThreads = 256;
    static constexpr int kWavesPerEu = 1;
    int64_t n;
    double L;
    double alpha;
    int n_split;
    const d4 *pq;
    const int *perm;
    const d4 *freal;
    const d4 *gpart;
    const double *scalars;
    const double *gscale;
    double *forces;
    double *dEdq;
    double *epart;
    __device__ void run(int bx, int by) const
    {
        final_p_body(bx, by, n, L, alpha, n_split, pq, perm, freal, gpart, scalars, gscale, forces, dEdq, epart);
    }
    hipError_t one(hipStream_t s, dim3 grid, int threads, size_t smem) const;
};

__global__ __launch_bounds__(256) void k_final_p(int64_t n, double L, double alpha, int n_split,
                                                 const d4 *__restrict__ pq, const int *__restrict__ perm,
                                                 const d4 *__restrict__ freal, const d4 *__restrict__ gpart,
                                                 const double *__restrict__ scalars, const double *__restrict__ gscale,
                                                 double *__restrict__ forces, double *__restrict__ dEdq,
                                                 double *__restrict__ epart)
{
    final_p_body(blockIdx.x, blockIdx.y, n, L, alpha, n_split, pq, perm, freal, gpart, scalars, gscale, forces, dEdq,
                 epart);
}

hipError_t KFinalP::one(hipStream_t s, dim3 grid, int threads, size_t smem) const
{
    hipLaunchKernelGGL((k_final_p), grid, dim3(threads), smem, s, n, L, alpha, n_split, pq, perm, freal, gpart, scalars,
                       gscale, forces, dEdq, epart);
    return hipGetLastError();
}

__device__ inline double ordered_block_sum(const double *__restrict__ v, int count, double *sh)
{
    const int t = threadIdx.x;
    const int per = (count + 255) / 256;
    double a = 0.0;
    for (int k = t * per; k < (t + 1) * per && k < count; ++k) a += v[k];
    sh[t] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Totals from the real-space block partials (epart) and the reciprocal ones
// (erec); thread 0 writes them.  status[0]: non-finite flag of this
// evaluation (set by the binning), latched into status[1] and cleared here.
__device__ inline void final_energy(int n_epart, const double *epart, int n_erec, const double *__restrict__ erec,
                                    double L, double alpha, const double *__restrict__ scalars,
                                    int *__restrict__ status, double *__restrict__ energy, double *sh)
{
    const double e_real = ordered_block_sum(epart, n_epart, sh);
    const double e_recip = ordered_block_sum(erec, n_erec, sh);
    if (threadIdx.x == 0) {
        const double V = L * L * L;
        const double Q = scalars[0];
        const double e_self = -sqrt(alpha / kPi) * scalars[1];
        const double e_bg = -kPi * Q * Q / (2.0 * V * alpha);
        double tot = e_real + e_recip + e_self + e_bg;
        const int bad = status[0];
        if (bad) {
            tot = __builtin_nan("");
            status[1] |= bad;
            status[0] = 0;
        }
        energy[0] = tot;
        energy[1] = e_real;
        energy[2] = e_recip;
        energy[3] = e_self;
        energy[4] = e_bg;
    }
}

__device__ __forceinline__ void final_e_body(int bx, int by, int n_epart, const double *__restrict__ epart, int n_erec,
                                             const double *__restrict__ erec, double L, double alpha,
                                             const double *__restrict__ scalars, int *__restrict__ status,
                                             double *__restrict__ energy)
{
    __shared__ double sh[256];
    final_energy(n_epart, epart, n_erec, erec, L, alpha, scalars, status, energy, sh);
}

struct KFinalE {
    static constexpr int kThreads = 256;
    static constexpr int kWavesPerEu = 1;
    int n_epart;
    const double *epart;
    int n_erec;
    const double *erec;
    double L;
    double alpha;
    const double *scalars;
    int *status;
    double *energy;
    __device__ void run(int bx, int by) const
    {
        final_e_body(bx, by, n_epart, epart, n_erec, erec, L, alpha, scalars, status, energy);
    }
    hipError_t one(hipStream_t s, dim3 grid, int threads, size_t smem) const;
};

__global__ __launch_bounds__(256) void k_final_e(int n_epart, const double *__restrict__ epart, int n_erec,
                                                 const double *__restrict__ erec, double L, double alpha,
                                                 const double *__restrict__ scalars, int *__restrict__ status,
                                                 double *__restrict__ energy)
{
    final_e_body(blockIdx.x, blockIdx.y, n_epart, epart, n_erec, erec, L, alpha, scalars, status, energy);
}

hipError_t KFinalE::one(hipStream_t s, dim3 grid, int threads, size_t smem) const
{
    hipLaunchKernelGGL((k_final_e), grid, dim3(threads), smem, s, n_epart, epart, n_erec, erec, L, alpha, scalars,
                       status, energy);
    return hipGetLastError();
}

// Both passes in one workgroup for n <= kSmallFinalMaxN: the blocks of k_final_p
// one after the other, their partials kept in LDS, then k_final_e; the same
// sums in the same order.
constexpr int kSmallFinalMaxN = 512;
__device__ __forceinline__ void final_small_body(int bx, int by, int64_t n, double L, double alpha, int n_split,
                                                 const d4 *__restrict__ pq, const int *__restrict__ perm,
                                                 const d4 *__restrict__ freal, const d4 *__restrict__ gpart,
                                                 const double *__restrict__ scalars, const double *__restrict__ gscale,
                                                 double *__restrict__ forces, double *__restrict__ dEdq, int n_erec,
                                                 const double *__restrict__ erec, int *__restrict__ status,
                                                 double *__restrict__ energy)
{
    __shared__ double s_e[256];
    __shared__ double s_part[kSmallFinalMaxN / 256];
    const int nb = (int)((n + 255) / 256);
    for (int b = 0; b < nb; ++b) {
        const int64_t s = (int64_t)b * 256 + threadIdx.x;
        s_e[threadIdx.x] = final_particle(s, n, L, alpha, n_split, pq, perm, freal, gpart, scalars, gscale, forces,
                                          dEdq);
        const double e = block_tree256(s_e);
        if (threadIdx.x == 0) s_part[b] = e;
        __syncthreads();  // s_e is refilled by the next block
    }
    __syncthreads();
    final_energy(nb, s_part, n_erec, erec, L, alpha, scalars, status, energy, s_e);
}

struct KFinalSmall {
    static constexpr int kThreads = 256;
    static constexpr int kWavesPerEu = 1;
    int64_t n;
    double L;
    double alpha;
    int n_split;
    const d4 *pq;
    const int *perm;
    const d4 *freal;
    const d4 *gpart;
    const double *scalars;
    const double *gscale;
    double *forces;
    double *dEdq;
    int n_erec;
    const double *erec;
    int *status;
    double *energy;
    __device__ void run(int bx, int by) const
    {
        final_small_body(bx, by, n, L, alpha, n_split, pq, perm, freal, gpart, scalars, gscale, forces, dEdq, n_erec,
                         erec, status, energy);
    }
    hipError_t one(hipStream_t s, dim3 grid, int threads, size_t smem) const;
};

__global__ __launch_bounds__(256) void k_final_small(int64_t n, double L, double alpha, int n_split,
                                                     const d4 *__restrict__ pq, const int *__restrict__ perm,
                                                     const d4 *__restrict__ freal, const d4 *__restrict__ gpart,
                                                     const double *__restrict__ scalars,
                                                     const double *__restrict__ gscale, double *__restrict__ forces,
                                                     double *__restrict__ dEdq, int n_erec,
                                                     const double *__restrict__ erec, int *__restrict__ status,
                                                     double *__restrict__ energy)
{
    final_small_body(blockIdx.x, blockIdx.y, n, L, alpha, n_split, pq, perm, freal, gpart, scalars, gscale, forces,
                     dEdq, n_erec, erec, status, energy);
}

hipError_t KFinalSmall::one(hipStream_t s, dim3 grid, int threads, size_t smem) const
{
    hipLaunchKernelGGL((k_final_small), grid, dim3(threads), smem, s, n, L, alpha, n_split, pq, perm, freal, gpart,
                       scalars, gscale, forces, dEdq, n_erec, erec, status, energy);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_finalize_particles(hipStream_t s, const FinalArgs &a, const d4 *pq, const int *perm,
                                     const d4 *freal, const d4 *gpart, const double *scalars, double *forces,
                                     double *dEdq, double *epart)
{
    return launch(s, dim3(ceil_div(a.n, 256)), 256, 0,
                  KFinalP{a.n, a.L, a.alpha, a.n_split, pq, perm, freal, gpart, scalars, a.gscale, forces, dEdq,
                          epart});
}

bool finalize_small(int64_t n) { return n <= kSmallFinalMaxN; }

hipError_t launch_finalize_small(hipStream_t s, const FinalArgs &a, const d4 *pq, const int *perm, const d4 *freal,
                                 const d4 *gpart, const double *scalars, double *forces, double *dEdq,
                                 const double *erec_part, const int *status, double *energy)
{
    return launch(s, dim3(1), 256, 0,
                  KFinalSmall{a.n, a.L, a.alpha, a.n_split, pq, perm, freal, gpart, scalars, a.gscale, forces, dEdq,
                              a.n_erec, erec_part, const_cast<int *>(status), energy});
}

hipError_t launch_finalize_energy(hipStream_t s, const FinalArgs &a, const double *epart, int n_epart,
                                  const double *erec_part, const double *scalars, const int *status,
                                  double *energy)
{
    return launch(s, dim3(1), 256, 0,
                  KFinalE{n_epart, epart, a.n_erec, erec_part, a.L, a.alpha, scalars, const_cast<int *>(status),
                          energy});
}

}  // namespace ewk
