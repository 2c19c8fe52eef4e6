// Non-periodic (isolated-system) QEq: the Coulomb operator between normalised
// Gaussian charges with no periodic images,
//   E_ij = erf(r_ij / (sqrt2 gamma_ij)) / r_ij,   E_ii = 1 / (sigma_i sqrt(pi)),
// (Electrostatics and Charge Equilibration section, the cases after eq.
// elec_energy), for molecules and clusters in several total-charge states.
// The product runs over all pairs (the direct solver of the Electrostatics
// Solvers section, O(N^2) per product, no grid and no cutoff); the projected
// CG loop and the energy / force epilogue are the periodic solve's.
//
// Layout: atoms stay in the caller's order (identity permutation); positions
// as double4 (x, y, z, sigma^2).  One product: blocks of 256 atoms i times
// atom splits over the j tiles; each tile of 256 atoms j is staged in LDS;
// the splits are added in a fixed order by the epilogue (deterministic).
// Differences of positions, squared distances, products with the source and
// all sums are FP64; the kernel values K(r) and K'(r)/r are FP32.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "internal.h"

namespace {

constexpr int NP_TILE = 256;
constexpr int NP_SPLIT_MAX = 64;
constexpr double NP_RSQPI = 0.56418958354775628695;   // 1/sqrt(pi)

// Validate, identity order, per-atom data; partial sums [sum chi, sum 1/D] in
// the layout the right-hand-side norm kernels read.
__global__ void k_np_stage(int n, const double* __restrict__ pos, const double* __restrict__ sigma,
                           const double* __restrict__ J, const double* __restrict__ chi, int* __restrict__ perm,
                           double4* __restrict__ npos, double* __restrict__ sig_s, double* __restrict__ J_s,
                           double* __restrict__ chi_s, double* __restrict__ chi_raw_s,
                           double* __restrict__ dself, double* __restrict__ dinv, double* __restrict__ part,
                           CgScalars* sc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double acc[2] = {0.0, 0.0};
    if (i < n) {
        const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
        const double sg = sigma[i], jj = J[i], c = chi[i];
        const bool ok = isfinite(x) && isfinite(y) && isfinite(z) && isfinite(c) && isfinite(sg) &&
                        isfinite(jj) && sg > 0.0 && jj > 0.0;
        if (!ok) atomicOr(&sc->err, QEQ_ERRBIT_INPUT);
        perm[i] = i;
        npos[i] = make_double4(x, y, z, sg * sg);
        sig_s[i] = sg;
        J_s[i] = jj;
        chi_s[i] = c;
        chi_raw_s[i] = c;
        dself[i] = NP_RSQPI / sg;
        dinv[i] = 1.0 / (jj + NP_RSQPI / sg);
        acc[0] = c;
        acc[1] = dinv[i];
    }
    block_sum<2>(acc);
    if (threadIdx.x == 0) {
        part[blockIdx.x * QEQ_NPART + 0] = acc[0];
        part[blockIdx.x * QEQ_NPART + 1] = acc[1];
    }
}

__global__ void k_np_zero(double* __restrict__ x, size_t m) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) x[i] = 0.0;
}

// K(r) and K'(r)/r for a = 1 / (sqrt2 gamma), x = a r.  Below x = 0.3 the
// Taylor series of erf(x)/x and of its derivative (the closed form of K'/r
// loses digits to cancellation there, and both are singular at r = 0).
__device__ __forceinline__ void np_kernel(float r2, float a, float& K, float& dKr) {
    const float r = sqrtf(r2);
    const float x = a * r;
    const float c = 1.12837916709551257390f * a;   // 2a / sqrt(pi)
    if (x < 0.3f) {
        const float x2 = x * x;
        K = c * (1.f + x2 * (-1.f / 3.f + x2 * (1.f / 10.f + x2 * (-1.f / 42.f + x2 * (1.f / 216.f)))));
        dKr = c * a * a *
              (-2.f / 3.f + x2 * (2.f / 5.f + x2 * (-1.f / 7.f + x2 * (1.f / 27.f + x2 * (-1.f / 132.f)))));
    } else {
        K = erff(x) / r;
        dKr = (c * __expf(-x * x) - K) / r2;
    }
}

// Partial products over the pair sum: ypart[split][i] = sum_{j in split, j != i}
// K_ij src_j; with FIN also fpart[split][i][c] = sum_j K'_ij / r_ij src_j (r_i - r_j)_c.
template <bool FIN>
__global__ __launch_bounds__(NP_TILE) void k_np_pairs(int n, int tiles_per_split, const double4* __restrict__ npos,
                                                      const double* __restrict__ src, double* __restrict__ ypart,
                                                      double* __restrict__ fpart, const int* __restrict__ done) {
    if (done && *done) return;
    __shared__ double4 pj[NP_TILE];
    __shared__ double sj[NP_TILE];
    const int i = blockIdx.x * NP_TILE + threadIdx.x;
    const int sp = blockIdx.y;
    const int ntiles = (n + NP_TILE - 1) / NP_TILE;
    const int t0 = sp * tiles_per_split, t1 = min(ntiles, t0 + tiles_per_split);
    const double4 pi = i < n ? npos[i] : make_double4(0.0, 0.0, 0.0, 1.0);
    const float si2 = (float)pi.w;
    double y = 0.0, g[3] = {0.0, 0.0, 0.0};
    for (int t = t0; t < t1; ++t) {
        const int j = t * NP_TILE + threadIdx.x;
        __syncthreads();
        // padded atoms far away with zero source: finite terms times zero
        pj[threadIdx.x] = j < n ? npos[j] : make_double4(1e10, 1e10, 1e10, 1.0);
        sj[threadIdx.x] = j < n ? src[j] : 0.0;
        __syncthreads();
        const int self = i - t * NP_TILE;   // in [0, NP_TILE) only on the diagonal tile
        for (int jj = 0; jj < NP_TILE; ++jj) {
            const double4 q = pj[jj];
            const double dx = pi.x - q.x, dy = pi.y - q.y, dz = pi.z - q.z;
            const float r2 = (float)(dx * dx + dy * dy + dz * dz);
            const float a = rsqrtf(2.f * (si2 + (float)q.w));
            float K, dKr;
            np_kernel(r2, a, K, dKr);
            const double s = jj == self ? 0.0 : sj[jj];
            y += (double)K * s;
            if (FIN) {
                const double w = (double)dKr * s;
                g[0] += w * dx;
                g[1] += w * dy;
                g[2] += w * dz;
            }
        }
    }
    if (i < n) {
        ypart[(size_t)sp * n + i] = y;
        if (FIN)
            for (int c = 0; c < 3; ++c) fpart[((size_t)sp * n + i) * 3 + c] = g[c];
    }
}

// Epilogue of one product, with the partial sums of the periodic path's
// matvec in the same slots: CG mode y = (E + diag J) src, slots [src.y, sum y];
// FINAL mode y = E src, forces -src_i sum_j ..., the gradient g = y + J q +
// chi and slots [q.E q, chi.q, J q^2, sigma^2 q, sum g].
template <int MODE>
__global__ void k_np_finish(int n, int nsplit, const double* __restrict__ src, const double* __restrict__ ypart,
                            const double* __restrict__ fpart, const double* __restrict__ dself,
                            const double* __restrict__ Jv, const double* __restrict__ chi_raw,
                            const double* __restrict__ chi_eff, const double* __restrict__ sig,
                            double* __restrict__ dst, double* __restrict__ forces, double* __restrict__ gvec,
                            double* __restrict__ part, const int* __restrict__ done) {
    if (MODE == QEQ_MODE_CG && done && *done) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (i < n) {
        const double vi = src[i];
        double y = dself[i] * vi;
        for (int sp = 0; sp < nsplit; ++sp) y += ypart[(size_t)sp * n + i];
        if (MODE == QEQ_MODE_CG) {
            y += Jv[i] * vi;
            acc[0] = vi * y;
            acc[1] = y;
        }
        dst[i] = y;
        if (MODE == QEQ_MODE_FINAL) {
            double g[3] = {0.0, 0.0, 0.0};
            for (int sp = 0; sp < nsplit; ++sp)
                for (int c = 0; c < 3; ++c) g[c] += fpart[((size_t)sp * n + i) * 3 + c];
            for (int c = 0; c < 3; ++c) forces[3 * i + c] = -vi * g[c];
            const double J = Jv[i];
            const double gi = y + J * vi + chi_eff[i];
            gvec[i] = gi;
            acc[0] = vi * y;
            acc[1] = chi_raw[i] * vi;
            acc[2] = J * vi * vi;
            acc[3] = sig[i] * sig[i] * vi;
            acc[4] = gi;
        }
    }
    if (MODE == QEQ_MODE_ELEC) return;   // uniform per launch: no partial sums
    block_sum<5>(acc);
    if (threadIdx.x == 0)
        for (int t = 0; t < 5; ++t) part[blockIdx.x * QEQ_NPART + t] = acc[t];
}

int np_alloc(double** p, size_t count) {
    *p = nullptr;
    if (hipMalloc((void**)p, sizeof(double) * (count ? count : 1)) != hipSuccess) return QEQ_ENOMEM;
    debug_poison(*p, sizeof(double) * count);
    return QEQ_OK;
}

}  // namespace

void np_free(qeq_plan* pl) {
    double* ptrs[] = {pl->np_pos, pl->np_ypart, pl->np_fpart};
    for (double* q : ptrs)
        if (q) (void)hipFree(q);
    pl->np_pos = pl->np_ypart = pl->np_fpart = nullptr;
    pl->np_cap = 0;
}

int np_setup(qeq_plan* pl, int n, const double* pos, const double* sigma, const double* J, const double* chi,
             double q_tot) {
    if (n < 1) return QEQ_EINVAL;
    if (n > pl->n_max) return QEQ_EPLAN;
    if (!isfinite(q_tot)) return QEQ_EINVAL;
    if (pl->np_cap < pl->n_max) {
        np_free(pl);
        const size_t m = (size_t)pl->n_max;
        QEQ_TRY(np_alloc(&pl->np_pos, 4 * m));   // double4 per atom
        QEQ_TRY(np_alloc(&pl->np_ypart, (size_t)NP_SPLIT_MAX * m));
        QEQ_TRY(np_alloc(&pl->np_fpart, (size_t)NP_SPLIT_MAX * m * 3));
        pl->np_cap = pl->n_max;
    }
    KParams& k = pl->kp;
    memset(&k, 0, sizeof(k));
    k.n = n;
    k.eta = pl->prm.eta;      // enters only through bg_pref = 0
    k.bg_pref = 0.0;          // no neutralising background: isolated system
    k.q_tot = q_tot;
    k.tol = pl->prm.tol;
    // atom splits: about 2048 blocks in all, each split a whole number of tiles
    const int ntiles = (n + NP_TILE - 1) / NP_TILE;
    int ns = std::max(1, std::min({NP_SPLIT_MAX, ntiles, (2048 + ntiles - 1) / ntiles}));
    pl->np_tps = (ntiles + ns - 1) / ns;
    pl->np_nsplit = (ntiles + pl->np_tps - 1) / pl->np_tps;
    QEQ_HIP(hipMemsetAsync(pl->sc, 0, sizeof(CgScalars), pl->stream));
    const int nb = nblocks(n);
    hipLaunchKernelGGL(k_np_stage, dim3(nb), dim3(QEQ_BLOCK), 0, pl->stream, n, pos, sigma, J, chi, pl->perm,
                       (double4*)pl->np_pos, pl->sig, pl->Jv, pl->chi, pl->chi_raw, pl->dself, pl->dinv, pl->part,
                       pl->sc);
    QEQ_TRY(qeq_check(hipGetLastError()));
    QEQ_TRY(launch_rhs_norm(pl, pl->chi));
    // the matvec partials fill the first nblocks(n) slots of the first partial
    // buffer; the CG kernels read interp_blocks(n) >= nblocks(n) of them
    const size_t m = (size_t)interp_blocks(n) * QEQ_NPART;
    hipLaunchKernelGGL(k_np_zero, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, pl->stream, pl->part, m);
    QEQ_HIP(hipMemcpyAsync(pl->sc_host, pl->sc, sizeof(CgScalars), hipMemcpyDeviceToHost, pl->stream));
    QEQ_HIP(hipStreamSynchronize(pl->stream));
    if (pl->sc_host->err & QEQ_ERRBIT_INPUT) return QEQ_EINVAL;
    return QEQ_OK;
}

int launch_np_matvec(qeq_plan* pl, const double* src, double* dst, int mode) {
    const int n = pl->kp.n;
    const int ntiles = (n + NP_TILE - 1) / NP_TILE;
    const dim3 grid(ntiles, pl->np_nsplit);
    const double4* npos = (const double4*)pl->np_pos;
    // QEQ_MODE_MATVEC: the CG product without the convergence flag (timing)
    const int* done = mode == QEQ_MODE_CG ? &pl->sc->done : nullptr;
    double* part = pl->part;
    if (mode == QEQ_MODE_FINAL) {
        hipLaunchKernelGGL(k_np_pairs<true>, grid, dim3(NP_TILE), 0, pl->stream, n, pl->np_tps, npos, src,
                           pl->np_ypart, pl->np_fpart, done);
        hipLaunchKernelGGL(k_np_finish<QEQ_MODE_FINAL>, dim3(nblocks(n)), dim3(QEQ_BLOCK), 0, pl->stream, n,
                           pl->np_nsplit, src, pl->np_ypart, pl->np_fpart, pl->dself, pl->Jv, pl->chi_raw, pl->chi,
                           pl->sig, dst, pl->fdst, pl->gtmp, part, done);
    } else if (mode == QEQ_MODE_ELEC) {
        hipLaunchKernelGGL(k_np_pairs<false>, grid, dim3(NP_TILE), 0, pl->stream, n, pl->np_tps, npos, src,
                           pl->np_ypart, pl->np_fpart, nullptr);
        hipLaunchKernelGGL(k_np_finish<QEQ_MODE_ELEC>, dim3(nblocks(n)), dim3(QEQ_BLOCK), 0, pl->stream, n,
                           pl->np_nsplit, src, pl->np_ypart, pl->np_fpart, pl->dself, pl->Jv, pl->chi_raw, pl->chi,
                           pl->sig, dst, pl->fdst, pl->gtmp, part, nullptr);
    } else {
        hipLaunchKernelGGL(k_np_pairs<false>, grid, dim3(NP_TILE), 0, pl->stream, n, pl->np_tps, npos, src,
                           pl->np_ypart, pl->np_fpart, done);
        hipLaunchKernelGGL(k_np_finish<QEQ_MODE_CG>, dim3(nblocks(n)), dim3(QEQ_BLOCK), 0, pl->stream, n,
                           pl->np_nsplit, src, pl->np_ypart, pl->np_fpart, pl->dself, pl->Jv, pl->chi_raw, pl->chi,
                           pl->sig, dst, pl->fdst, pl->gtmp, part, done);
    }
    return qeq_check(hipGetLastError());
}
