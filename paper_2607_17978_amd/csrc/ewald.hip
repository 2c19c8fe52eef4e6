// Reciprocal part of the periodic operator by direct Ewald summation (SI,
// "Ewald Summation"; the Electrostatics Solvers section's O(N^3/2) solver for
// small cells), in place of the particle mesh:
//
//   (E_rec v)_i = sum_{k in a half space, 0 < |k| <= k_max} w_k
//                 [cos(k.r_i) C_k + sin(k.r_i) S_k],
//   C_k + i S_k = sum_j v_j exp(i k.r_j),   w_k = 2 (4 pi / V) exp(-eta^2 k^2 / 2) / k^2,
//
// with k = 2 pi H^-1 m and k_max where exp(-eta^2 k^2 / 2) = 1e-12.  The
// real-space pairs, the self and background terms and the CG loop are the
// mesh path's (the mesh self-correction is off: the sums are exact).  Forces
// of the final product: F_i = -q_i sum_k w_k k [S_k cos(k.r_i) - C_k sin(k.r_i)].
//
// Two passes per product, both O(N M) phase evaluations: structure factors
// (thread per mode, atoms staged in LDS, atom splits) and the potential
// (thread per atom, modes staged in LDS with their k vectors, mode splits),
// then a fixed-order sum of the splits (deterministic).  Phases: the argument
// m.s in FP64 reduced to one turn, sin/cos in FP32; sums in FP64.
#include <math.h>

#include <algorithm>
#include <vector>

#include "internal.h"

namespace {

constexpr int EW_T = 256;            // threads per block
constexpr int EW_MAX_MODES = 1 << 20;
constexpr int EW_SPLIT_MAX = 64;
constexpr double EW_PI = 3.14159265358979323846;

// Structure-factor partials: block (256 modes, atom split).
__global__ __launch_bounds__(EW_T) void k_ew_sf(int n, int nm, int per, const int4* __restrict__ modes,
                                                const double* __restrict__ frac, const double* __restrict__ src,
                                                double* __restrict__ sfpart, const int* __restrict__ done) {
    if (done && *done) return;
    __shared__ double ss[EW_T][4];
    const int m = blockIdx.x * EW_T + threadIdx.x;
    const int sp = blockIdx.y;
    const int i0 = sp * per, i1 = min(n, i0 + per);
    int4 md = make_int4(0, 0, 0, 0);
    if (m < nm) md = modes[m];
    double C = 0.0, S = 0.0;
    for (int c0 = i0; c0 < i1; c0 += EW_T) {
        __syncthreads();
        const int i = c0 + threadIdx.x;
        if (i < i1) {
            ss[threadIdx.x][0] = frac[3 * i];
            ss[threadIdx.x][1] = frac[3 * i + 1];
            ss[threadIdx.x][2] = frac[3 * i + 2];
            ss[threadIdx.x][3] = src[i];
        }
        __syncthreads();
        const int cnt = min(EW_T, i1 - c0);
        for (int a = 0; a < cnt; ++a) {
            double t = (double)md.x * ss[a][0] + (double)md.y * ss[a][1] + (double)md.z * ss[a][2];
            t -= rint(t);
            float sn, cs;
            sincospif(2.0f * (float)t, &sn, &cs);
            C += ss[a][3] * (double)cs;
            S += ss[a][3] * (double)sn;
        }
    }
    if (m < nm) {
        sfpart[((size_t)sp * nm + m) * 2] = C;
        sfpart[((size_t)sp * nm + m) * 2 + 1] = S;
    }
}

// Potential (and with FIN the force sums) of each atom from one range of
// modes: block (256 atoms, mode split).  ypart[split][i], fpart[split][i][3].
template <bool FIN>
__global__ __launch_bounds__(EW_T) void k_ew_pot(int n, int nm, int mper, int fs, KParams k,
                                                 const int4* __restrict__ modes, const double* __restrict__ wk,
                                                 const double* __restrict__ frac, const double* __restrict__ sfpart,
                                                 double* __restrict__ ypart, double* __restrict__ fpart,
                                                 const int* __restrict__ done) {
    if (done && *done) return;
    __shared__ int4 ms[EW_T];
    __shared__ double wc[EW_T], wsn[EW_T];
    __shared__ float kv[EW_T][3];
    const int i = blockIdx.x * EW_T + threadIdx.x;
    const int sp = blockIdx.y;
    const int m0 = sp * mper, m1 = min(nm, m0 + mper);
    double s[3] = {0.0, 0.0, 0.0};
    if (i < n) {
        s[0] = frac[3 * i];
        s[1] = frac[3 * i + 1];
        s[2] = frac[3 * i + 2];
    }
    double y = 0.0, f[3] = {0.0, 0.0, 0.0};
    for (int c0 = m0; c0 < m1; c0 += EW_T) {
        __syncthreads();
        const int m = c0 + threadIdx.x;
        if (m < m1) {
            const int4 md = modes[m];
            double C = 0.0, S = 0.0;
            for (int q = 0; q < fs; ++q) {
                C += sfpart[((size_t)q * nm + m) * 2];
                S += sfpart[((size_t)q * nm + m) * 2 + 1];
            }
            ms[threadIdx.x] = md;
            wc[threadIdx.x] = wk[m] * C;
            wsn[threadIdx.x] = wk[m] * S;
            if (FIN) {
                // k = 2 pi H^-1 m (Cartesian), column convention of the cell rows
                for (int c = 0; c < 3; ++c)
                    kv[threadIdx.x][c] = (float)(2.0 * EW_PI *
                                                 (k.Hinv[c * 3] * md.x + k.Hinv[c * 3 + 1] * md.y +
                                                  k.Hinv[c * 3 + 2] * md.z));
            }
        }
        __syncthreads();
        const int cnt = min(EW_T, m1 - c0);
        for (int a = 0; a < cnt; ++a) {
            const int4 md = ms[a];
            double t = (double)md.x * s[0] + (double)md.y * s[1] + (double)md.z * s[2];
            t -= rint(t);
            float sn, cs;
            sincospif(2.0f * (float)t, &sn, &cs);
            y += wc[a] * (double)cs + wsn[a] * (double)sn;
            if (FIN) {
                const double g = wsn[a] * (double)cs - wc[a] * (double)sn;
                f[0] += g * (double)kv[a][0];
                f[1] += g * (double)kv[a][1];
                f[2] += g * (double)kv[a][2];
            }
        }
    }
    if (i < n) {
        ypart[(size_t)sp * n + i] = y;
        if (FIN)
            for (int c = 0; c < 3; ++c) fpart[((size_t)sp * n + i) * 3 + c] = f[c];
    }
}

// yrec[i] = sum of the mode splits; with FIN also the forces of the
// reciprocal part, frec_i = -q_i sum f (added to the pair forces afterwards).
template <bool FIN>
__global__ void k_ew_sum(int n, int ms, const double* __restrict__ ypart, const double* __restrict__ fpart,
                         const double* __restrict__ src, double* __restrict__ yrec, double* __restrict__ frec,
                         const int* __restrict__ done) {
    if (done && *done) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double y = 0.0;
    for (int q = 0; q < ms; ++q) y += ypart[(size_t)q * n + i];
    yrec[i] = y;
    if (FIN) {
        double f[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < ms; ++q)
            for (int c = 0; c < 3; ++c) f[c] += fpart[((size_t)q * n + i) * 3 + c];
        for (int c = 0; c < 3; ++c) frec[3 * i + c] = -src[i] * f[c];
    }
}

__global__ void k_ew_add_forces(int n, const double* __restrict__ frec, double* __restrict__ forces) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 3 * n) forces[t] += frec[t];
}

template <typename T>
int ew_alloc(T** p, size_t count) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    if (hipMalloc((void**)p, sizeof(T) * (count ? count : 1)) != hipSuccess) return QEQ_ENOMEM;
    if (poisonable<T>) debug_poison(*p, sizeof(T) * count);
    return QEQ_OK;
}

}  // namespace

void ew_free(qeq_plan* pl) {
    void* ptrs[] = {pl->ew_modes, pl->ew_w, pl->ew_sf, pl->ew_y, pl->ew_f, pl->ew_yrec, pl->ew_frec};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    pl->ew_modes = nullptr;
    pl->ew_w = pl->ew_sf = pl->ew_y = pl->ew_f = pl->ew_yrec = pl->ew_frec = nullptr;
    pl->ew_cap_m = pl->ew_cap_n = 0;
}

// Mode list of the current cell (half space, 0 < |k| <= k_max) and the split
// shapes; buffers grown as needed.
int ew_setup(qeq_plan* pl) {
    const KParams& k = pl->kp;
    const double eta = k.eta;
    const double kmax2 = 2.0 * log(1e12) / (eta * eta);
    int lim[3];
    for (int a = 0; a < 3; ++a) {
        const double len = sqrt(k.H[a * 3] * k.H[a * 3] + k.H[a * 3 + 1] * k.H[a * 3 + 1] +
                                k.H[a * 3 + 2] * k.H[a * 3 + 2]);
        lim[a] = (int)ceil(sqrt(kmax2) * len / (2.0 * EW_PI)) + 1;
    }
    std::vector<int4> mm;
    std::vector<double> w;
    for (int m1 = 0; m1 <= lim[0]; ++m1)
        for (int m2 = -lim[1]; m2 <= lim[1]; ++m2)
            for (int m3 = -lim[2]; m3 <= lim[2]; ++m3) {
                if (m1 == 0 && (m2 < 0 || (m2 == 0 && m3 <= 0))) continue;
                double kv[3];
                for (int c = 0; c < 3; ++c)
                    kv[c] = 2.0 * EW_PI * (k.Hinv[c * 3] * m1 + k.Hinv[c * 3 + 1] * m2 + k.Hinv[c * 3 + 2] * m3);
                const double k2 = kv[0] * kv[0] + kv[1] * kv[1] + kv[2] * kv[2];
                if (k2 > kmax2) continue;
                mm.push_back(make_int4(m1, m2, m3, 0));
                w.push_back(2.0 * 4.0 * EW_PI / k.vol * exp(-0.5 * eta * eta * k2) / k2);
                if ((int)mm.size() > EW_MAX_MODES) return QEQ_EPLAN;   // cell too large for direct sums
            }
    const int nm = (int)mm.size();
    const int n = k.n;
    // splits: about 1024 blocks per pass, at least 64 atoms / 256 modes each
    const int mb = (nm + EW_T - 1) / EW_T, ab = (n + EW_T - 1) / EW_T;
    const int fs = std::max(1, std::min({EW_SPLIT_MAX, (1024 + mb - 1) / mb, std::max(1, n / 64)}));
    const int ms = std::max(1, std::min({EW_SPLIT_MAX, (1024 + ab - 1) / ab, std::max(1, nm / 256)}));
    if (nm > pl->ew_cap_m) {
        QEQ_TRY(ew_alloc((int4**)&pl->ew_modes, (size_t)nm));
        QEQ_TRY(ew_alloc(&pl->ew_w, (size_t)nm));
        QEQ_TRY(ew_alloc(&pl->ew_sf, (size_t)EW_SPLIT_MAX * nm * 2));
        pl->ew_cap_m = nm;
    }
    if (pl->n_max > pl->ew_cap_n) {
        const size_t nn = (size_t)pl->n_max;
        QEQ_TRY(ew_alloc(&pl->ew_y, (size_t)EW_SPLIT_MAX * nn));
        QEQ_TRY(ew_alloc(&pl->ew_f, (size_t)EW_SPLIT_MAX * nn * 3));
        QEQ_TRY(ew_alloc(&pl->ew_yrec, nn));
        QEQ_TRY(ew_alloc(&pl->ew_frec, nn * 3));
        pl->ew_cap_n = pl->n_max;
    }
    pl->ew_nm = nm;
    pl->ew_fs = fs;
    pl->ew_fper = (n + fs - 1) / fs;
    pl->ew_ms = ms;
    pl->ew_mper = (nm + ms - 1) / ms;
    if (nm > 0) {
        QEQ_HIP(hipMemcpyAsync(pl->ew_modes, mm.data(), sizeof(int4) * nm, hipMemcpyHostToDevice, pl->stream));
        QEQ_HIP(hipMemcpyAsync(pl->ew_w, w.data(), sizeof(double) * nm, hipMemcpyHostToDevice, pl->stream));
        QEQ_HIP(hipStreamSynchronize(pl->stream));   // the host vectors go out of scope
    }
    return QEQ_OK;
}

// yrec = E_rec src (sorted order); with fin also frec, the reciprocal forces
// (added to the pair forces by launch_ew_forces_add after the final pass).
int launch_ew_rec(qeq_plan* pl, const double* src, const int* done, bool fin) {
    const int n = pl->kp.n, nm = pl->ew_nm;
    if (nm == 0) {
        // no reciprocal vector below the cutoff: the sums vanish
        if (fin)
            hipLaunchKernelGGL(k_ew_sum<true>, dim3(nblocks(n)), dim3(QEQ_BLOCK), 0, pl->stream, n, 0, pl->ew_y,
                               pl->ew_f, src, pl->ew_yrec, pl->ew_frec, done);
        else
            hipLaunchKernelGGL(k_ew_sum<false>, dim3(nblocks(n)), dim3(QEQ_BLOCK), 0, pl->stream, n, 0, pl->ew_y,
                               pl->ew_f, src, pl->ew_yrec, pl->ew_frec, done);
        return qeq_check(hipGetLastError());
    }
    hipLaunchKernelGGL(k_ew_sf, dim3((nm + EW_T - 1) / EW_T, pl->ew_fs), dim3(EW_T), 0, pl->stream, n, nm,
                       pl->ew_fper, (const int4*)pl->ew_modes, pl->frac, src, pl->ew_sf, done);
    const dim3 gp((n + EW_T - 1) / EW_T, pl->ew_ms);
    if (fin) {
        hipLaunchKernelGGL(k_ew_pot<true>, gp, dim3(EW_T), 0, pl->stream, n, nm, pl->ew_mper, pl->ew_fs, pl->kp,
                           (const int4*)pl->ew_modes, pl->ew_w, pl->frac, pl->ew_sf, pl->ew_y, pl->ew_f, done);
        hipLaunchKernelGGL(k_ew_sum<true>, dim3(nblocks(n)), dim3(QEQ_BLOCK), 0, pl->stream, n, pl->ew_ms, pl->ew_y,
                           pl->ew_f, src, pl->ew_yrec, pl->ew_frec, done);
    } else {
        hipLaunchKernelGGL(k_ew_pot<false>, gp, dim3(EW_T), 0, pl->stream, n, nm, pl->ew_mper, pl->ew_fs, pl->kp,
                           (const int4*)pl->ew_modes, pl->ew_w, pl->frac, pl->ew_sf, pl->ew_y, pl->ew_f, done);
        hipLaunchKernelGGL(k_ew_sum<false>, dim3(nblocks(n)), dim3(QEQ_BLOCK), 0, pl->stream, n, pl->ew_ms,
                           pl->ew_y, pl->ew_f, src, pl->ew_yrec, pl->ew_frec, done);
    }
    return qeq_check(hipGetLastError());
}

int launch_ew_forces_add(qeq_plan* pl) {
    const int n = pl->kp.n;
    hipLaunchKernelGGL(k_ew_add_forces, dim3(nblocks(3 * n)), dim3(QEQ_BLOCK), 0, pl->stream, n, pl->ew_frec,
                       pl->fdst);
    return qeq_check(hipGetLastError());
}
