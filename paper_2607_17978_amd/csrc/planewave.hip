// Gaussian-on-grid ("plane-wave") Coulomb operator: the matrix-vector
// product of the paper's eq. matvec evaluated without an Ewald split
// ("Electrostatics Solvers": the charge density is put on a uniform grid,
// Fourier transformed, multiplied by 4 pi / G^2 and transformed back, and the
// potential is integrated over each atom's Gaussian density).
//
//   theta_i(g) = dV rho_i(r_g - r_i)
//              = dV / ((2 pi)^{3/2} sigma_i^3) exp(-|r_g - r_i|^2 / (2 sigma_i^2)),
//   Q(g)       = sum_j src_j theta_j(g)                  (all periodic images)
//   phi        = unnormalised inverse DFT of (4 pi / (V k^2)) DFT(Q), k != 0
//   (A src)_i  = sum_g theta_i(g) phi(g)
//   F_i        = -q_i sum_g theta_i(g) phi(g) (r_g - r_i) / sigma_i^2
//
// theta_i is cut at |r_g - r_i| <= c sigma_i (c = 6 by default: the
// discarded tail changes the operator by ~1e-8 relative at the configs'
// grid spacing).  With the k = 0 term omitted this is the plane-wave
// definition of the periodic Gaussian-charge energy, self interaction and
// neutralising background included, so there is no real-space pair term, no
// self term and no background correction.
//
// Passes per product:
//   1. zero the real grid; 2. spread, one wave per atom, FP32 global atomic
//   additions (the support of ~10^3-10^4 points per atom does not fit the
//   LDS tiles of the spline spread); 3. R2C along axis 3 in LDS tiles;
//   4. the spline path's axis-2 / axis-1 (+ Green's function with eta = 0
//   and unit moduli) / inverse passes; 5. integration, one wave per atom.
// Inside a wave the points of one grid plane of the support ellipsoid's
// bounding box are spread over the lanes with an incremental (row, column)
// counter, so that no lane divides per point.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "internal.h"

namespace {

constexpr int PW_NT = 256;
constexpr double PW_PI = 3.14159265358979323846;
constexpr float PW_LOG2E = 1.4426950408889634f;

__device__ __forceinline__ int pw_wrap(int g, int K) {
    if (g >= 0 && g < K) return g;
    const int m = g % K;
    return m < 0 ? m + K : m;
}

// Cross-section of the ellipsoid d^T G d <= R2 with the grid plane at offset
// d1 along axis 1: centre (x2, x3) and half-extents (e2, e3) of its bounding
// box; false when the plane misses it.  (The 2x2 block of G and the extent
// factors are constants of the cell, precomputed on the host.)
__device__ __forceinline__ bool pw_section(const PwGeom& g, float d1, float R2, float& x2, float& x3, float& e2,
                                           float& e3) {
    const float b2 = g.G[3] * d1, b3 = g.G[4] * d1;
    x2 = -(g.G[2] * b2 - g.G[5] * b3) * g.inv_det23;
    x3 = -(g.G[1] * b3 - g.G[5] * b2) * g.inv_det23;
    const float rho2 = R2 - (g.G[0] * d1 * d1 + b2 * x2 + b3 * x3);
    if (!(rho2 >= 0.f)) return false;
    const float rho = sqrtf(rho2);
    e2 = rho * g.ext2;
    e3 = rho * g.ext3;
    return true;
}

// Per-atom constants: integer cell of the atom on the grid, fractional offset
// inside it, and the Gaussian's parameters.
struct PwAtom {
    int fl[3];
    float du[3];
    float R2;    // (c sigma)^2 in bohr^2
    float lsc;   // log2(e) / (2 sigma^2)
};

__device__ __forceinline__ PwAtom pw_atom(const KParams& k, const PwGeom& g, const double* frac, double s, int i) {
    PwAtom a;
    const int Kd[3] = {k.K1, k.K2, k.K3};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double u = frac[3 * i + c] * (double)Kd[c];
        const double f = floor(u);
        a.fl[c] = (int)f;
        a.du[c] = (float)(u - f);
    }
    a.R2 = g.c2 * (float)(s * s);
    a.lsc = PW_LOG2E / (float)(2.0 * s * s);
    // a position the input check rejected: no support (the solve reports EINVAL)
    if (!(isfinite(a.du[0]) && isfinite(a.du[1]) && isfinite(a.du[2]) && a.R2 > 0.f)) {
        a.fl[0] = a.fl[1] = a.fl[2] = 0;
        a.du[0] = a.du[1] = a.du[2] = 0.f;
        a.R2 = 0.f;
    }
    return a;
}

// Walks the support of one atom plane by plane: body(idx, Q, d1, d2, d3) runs
// for every grid point inside the cut sphere (grid index, squared distance
// d^T G d, offsets in grid steps), the points spread over the lanes.
template <typename Body>
__device__ __forceinline__ void pw_walk(const KParams& k, const PwGeom& g, const PwAtom& a, int lane, Body body) {
    if (!(a.R2 > 0.f)) return;
    const float e1 = sqrtf(a.R2) * g.ext1;
    const int t1lo = (int)ceilf(a.du[0] - e1), t1hi = (int)floorf(a.du[0] + e1);
    for (int t1 = t1lo; t1 <= t1hi; ++t1) {
        const float d1 = (float)t1 - a.du[0];
        float x2, x3, e2, e3;
        if (!pw_section(g, d1, a.R2, x2, x3, e2, e3)) continue;
        const int t2lo = (int)ceilf(x2 - e2 + a.du[1]), t2hi = (int)floorf(x2 + e2 + a.du[1]);
        const int t3lo = (int)ceilf(x3 - e3 + a.du[2]), t3hi = (int)floorf(x3 + e3 + a.du[2]);
        const int n2 = t2hi - t2lo + 1, n3 = t3hi - t3lo + 1;
        if (n2 <= 0 || n3 <= 0) continue;
        const size_t pbase = (size_t)pw_wrap(a.fl[0] + t1, k.K1) * k.K2 * k.K3;
        const float c1 = g.G[0] * d1 * d1, l2 = 2.f * g.G[3] * d1, l3 = 2.f * g.G[4] * d1;
        const int nbox = n2 * n3;
        const int dq = 64 / n3, dr = 64 - dq * n3;
        // lane / n3 through the reciprocal: exact for lane < 64 (the quotient
        // is at least 0.5 / n3 away from an integer)
        int qq = (int)(((float)lane + 0.5f) * (1.0f / (float)n3));
        int rr = lane - qq * n3;
        for (int j = lane; j < nbox; j += 64) {
            const int t2 = t2lo + qq, t3 = t3lo + rr;
            const float d2 = (float)t2 - a.du[1], d3 = (float)t3 - a.du[2];
            const float Q = c1 + d2 * (l2 + g.G[1] * d2 + 2.f * g.G[5] * d3) + d3 * (l3 + g.G[2] * d3);
            if (Q <= a.R2) {
                const size_t idx = pbase + (size_t)pw_wrap(a.fl[1] + t2, k.K2) * k.K3 + pw_wrap(a.fl[2] + t3, k.K3);
                body(idx, Q, d1, d2, d3);
            }
            qq += dq;
            rr += dr;
            if (rr >= n3) {
                rr -= n3;
                ++qq;
            }
        }
    }
}

__global__ __launch_bounds__(PW_NT) void k_pw_zero(float4* __restrict__ grid, size_t n4, const int* __restrict__ done) {
    if (done && *done) return;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n4) grid[t] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// Q(g) += src_i theta_i(g), one wave per atom (sorted order).
__global__ __launch_bounds__(PW_NT) void k_pw_spread(KParams k, PwGeom g, const double* __restrict__ src,
                                                   const double* __restrict__ frac, const double* __restrict__ sig,
                                                   float* __restrict__ grid, const int* __restrict__ done) {
    if (done && *done) return;
    const int lane = threadIdx.x & 63;
    const int nwaves = gridDim.x * (PW_NT / 64);
    const int w0 = (xcd_remap(blockIdx.x, gridDim.x) * PW_NT + threadIdx.x) >> 6;
    for (int i = w0; i < k.n; i += nwaves) {
        const double q = src[i];
        if (q == 0.0) continue;
        const double s = sig[i];
        const PwAtom a = pw_atom(k, g, frac, s, i);
        const float amp = (float)(q * (double)g.wpref / (s * s * s));
        pw_walk(k, g, a, lane, [&](size_t idx, float Q, float, float, float) {
            unsafeAtomicAdd(grid + idx, amp * __builtin_amdgcn_exp2f(-Q * a.lsc));
        });
    }
}

// Axis-3 FFT of the tile in LDS (two real rows packed per complex column,
// acc[g3][row] viewed as buf[g3][row pair]) and the half spectra written
// transposed, C[m3][g1][g2] (m2 contiguous).
__device__ __forceinline__ void pw_tile_r2c(const KParams& k, const FftAxis& ax3, float2* buf, const float2* tw,
                                            int g1, int g20, float2* __restrict__ C, int tid) {
    const int K1 = k.K1, K2 = k.K2, K3 = k.K3, TW = k.TW, ncol = TW >> 1;
    int twl = 0;
    while ((1 << twl) < TW) ++twl;
    fft_lds(buf, ax3, twl - 1, tw, false, tid, PW_NT);
    __syncthreads();
    const int K3h = K3 / 2 + 1;
    for (int t = tid; t < K3h * TW; t += PW_NT) {
        const int r = t & (TW - 1);
        const int m = t >> twl;
        const int pr = r >> 1;
        const float2 Z = buf[m * ncol + pr];
        float2 Zc = buf[(m == 0 ? 0 : K3 - m) * ncol + pr];
        Zc.y = -Zc.y;
        float2 X;
        if ((r & 1) == 0) {
            X = make_float2(0.5f * (Z.x + Zc.x), 0.5f * (Z.y + Zc.y));
        } else {
            const float2 d = csub(Z, Zc);
            X = make_float2(0.5f * d.y, -0.5f * d.x);
        }
        C[((size_t)m * K1 + g1) * K2 + g20 + r] = X;
    }
}

// Real-to-complex transform along axis 3 of the real grid, block = (g1, tile
// of TW rows g2: the axis-1 / complex-to-real tile, a power of two), two
// real rows packed into one complex column; the half
// spectra are written transposed (C[m3][g1][g2]) as by the spline spread.
__global__ __launch_bounds__(PW_NT) void k_pw_r2c(KParams k, FftAxis ax3, const float* __restrict__ R,
                                                float2* __restrict__ C, const int* __restrict__ done) {
    if (done && *done) return;
    extern __shared__ float2 sm[];
    const int K2 = k.K2, K3 = k.K3, TW = k.TW;
    float2* tw = sm;
    float2* buf = sm + K3;
    float* acc = reinterpret_cast<float*>(buf);
    const int tid = threadIdx.x;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int g1 = blk / k.ntile;
    const int g20 = (blk - g1 * k.ntile) * TW;
    for (int t = tid; t < K3; t += PW_NT) tw[t] = ax3.tw[t];
    // row index fastest: consecutive lanes write consecutive LDS words (the
    // transposed [g3][row] layout the FFT needs); each lane loads 4 values
    // of its row (K3 % 4 == 0)
    for (int e = tid; e < TW * (K3 >> 2); e += PW_NT) {
        const int r = e & (TW - 1), c4 = e / TW;
        const float4 x = *reinterpret_cast<const float4*>(R + ((size_t)g1 * K2 + g20 + r) * K3 + 4 * c4);
        acc[(4 * c4) * TW + r] = x.x;
        acc[(4 * c4 + 1) * TW + r] = x.y;
        acc[(4 * c4 + 2) * TW + r] = x.z;
        acc[(4 * c4 + 3) * TW + r] = x.w;
    }
    __syncthreads();
    pw_tile_r2c(k, ax3, buf, tw, g1, g20, C, tid);
}

// y_i = sum_g theta_i(g) phi(g); with FIN the forces of that product for the
// charges src (both sorted order), one wave per atom.
template <bool FIN>
__global__ __launch_bounds__(PW_NT) void k_pw_interp(KParams k, PwGeom g, const double* __restrict__ src,
                                                   const double* __restrict__ frac, const double* __restrict__ sig,
                                                   const float* __restrict__ grid, double* __restrict__ y,
                                                   double* __restrict__ f, const int* __restrict__ done) {
    if (done && *done) return;
    const int lane = threadIdx.x & 63;
    const int nwaves = gridDim.x * (PW_NT / 64);
    const int w0 = (xcd_remap(blockIdx.x, gridDim.x) * PW_NT + threadIdx.x) >> 6;
    const int rounds = (k.n + nwaves - 1) / nwaves;
    for (int rnd = 0; rnd < rounds; ++rnd) {
        const int i = rnd * nwaves + w0;
        float v[4] = {0.f, 0.f, 0.f, 0.f};
        double s = 1.0;
        if (i < k.n) {
            s = sig[i];
            const PwAtom a = pw_atom(k, g, frac, s, i);
            pw_walk(k, g, a, lane, [&](size_t idx, float Q, float d1, float d2, float d3) {
                const float t = __builtin_amdgcn_exp2f(-Q * a.lsc) * grid[idx];
                v[0] += t;
                if (FIN) {
                    v[1] += t * d1;
                    v[2] += t * d2;
                    v[3] += t * d3;
                }
            });
        }
        double vd[4] = {(double)v[0], 0.0, 0.0, 0.0};
        vd[0] = wave_sum(vd[0]);
        if (FIN) {
#pragma unroll
            for (int c = 1; c < 4; ++c) vd[c] = wave_sum((double)v[c]);
        }
        if (i < k.n && lane == 0) {
            const double amp = (double)g.wpref / (s * s * s);
            y[i] = amp * vd[0];
            if (FIN) {
                // F = -q / sigma^2 sum theta phi (r_g - r_i), r_g - r_i = sum_a d_a H[a] / K_a
                const double pre = -src[i] * amp / (s * s);
                for (int c = 0; c < 3; ++c)
                    f[3 * i + c] = pre * (vd[1] * g.HK[c] + vd[2] * g.HK[3 + c] + vd[3] * g.HK[6 + c]);
            }
        }
    }
}

__global__ void k_pw_add_forces(int n, const double* __restrict__ frec, double* __restrict__ forces) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 3 * n) forces[t] += frec[t];
}

__global__ __launch_bounds__(PW_NT) void k_pw_sigma_max(int n, const double* __restrict__ sig,
                                                      double* __restrict__ part) {
    __shared__ double sh[PW_NT];
    const int i = blockIdx.x * PW_NT + threadIdx.x;
    sh[threadIdx.x] = i < n ? sig[i] : 0.0;
    __syncthreads();
    for (int w = PW_NT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

template <typename T>
int pw_alloc(T** p, size_t count) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    if (hipMalloc((void**)p, sizeof(T) * (count ? count : 1)) != hipSuccess) return QEQ_ENOMEM;
    if (poisonable<T>) debug_poison(*p, sizeof(T) * count);
    return QEQ_OK;
}

int pw_blocks(int n) {
    const int waves = PW_NT / 64;
    const int b = (n + waves - 1) / waves;
    return std::max(1, std::min(b, 2048));
}

bool invert3(const double m[9], double out[9]) {
    const double c00 = m[4] * m[8] - m[5] * m[7], c01 = m[5] * m[6] - m[3] * m[8], c02 = m[3] * m[7] - m[4] * m[6];
    const double det = m[0] * c00 + m[1] * c01 + m[2] * c02;
    if (!(fabs(det) > 0.0)) return false;
    const double id = 1.0 / det;
    out[0] = c00 * id;
    out[1] = (m[2] * m[7] - m[1] * m[8]) * id;
    out[2] = (m[1] * m[5] - m[2] * m[4]) * id;
    out[3] = c01 * id;
    out[4] = (m[0] * m[8] - m[2] * m[6]) * id;
    out[5] = (m[2] * m[3] - m[0] * m[5]) * id;
    out[6] = c02 * id;
    out[7] = (m[1] * m[6] - m[0] * m[7]) * id;
    out[8] = (m[0] * m[4] - m[1] * m[3]) * id;
    return true;
}

}  // namespace

void pw_free(qeq_plan* pl) {
    void* ptrs[] = {pl->pw_ones, pl->pw_y, pl->pw_f, pl->pw_smax};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    pl->pw_ones = nullptr;
    pl->pw_y = pl->pw_f = pl->pw_smax = nullptr;
    pl->pw_cap_n = pl->pw_cap_k = 0;
}

// Geometry of the current cell and grid; buffers grown as needed.  One host
// sync (the largest sigma bounds the support, checked against the grid).
int pw_setup(qeq_plan* pl) {
    const KParams& k = pl->kp;
    const int kmax = std::max({k.K1, k.K2, k.K3});
    if (kmax > pl->pw_cap_k) {
        QEQ_TRY(pw_alloc(&pl->pw_ones, (size_t)kmax));
        std::vector<float> ones((size_t)kmax, 1.0f);
        QEQ_HIP(hipMemcpy(pl->pw_ones, ones.data(), sizeof(float) * kmax, hipMemcpyHostToDevice));
        pl->pw_cap_k = kmax;
    }
    if (pl->n_max > pl->pw_cap_n) {
        const size_t nn = (size_t)pl->n_max;
        QEQ_TRY(pw_alloc(&pl->pw_y, nn));
        QEQ_TRY(pw_alloc(&pl->pw_f, 3 * nn));
        QEQ_TRY(pw_alloc(&pl->pw_smax, (nn + PW_NT - 1) / PW_NT));
        pl->pw_cap_n = pl->n_max;
    }
    const int Kd[3] = {k.K1, k.K2, k.K3};
    double G[9], Gi[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double d = 0.0;
            for (int c = 0; c < 3; ++c) d += k.H[a * 3 + c] * k.H[b * 3 + c];
            G[a * 3 + b] = d / ((double)Kd[a] * Kd[b]);
        }
    if (!invert3(G, Gi)) return QEQ_EINVAL;
    PwGeom& g = pl->pw_geom;
    const int o[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
    for (int t = 0; t < 6; ++t) g.G[t] = (float)G[o[t][0] * 3 + o[t][1]];
    // extent of d^T G d <= 1 along axis a: sqrt((G^-1)_aa); plane sections
    // use the inverse of the (2, 3) block of G
    const double det23 = G[4] * G[8] - G[5] * G[7];
    g.ext1 = (float)sqrt(Gi[0]);
    g.inv_det23 = (float)(1.0 / det23);
    g.ext2 = (float)sqrt(G[8] / det23);
    g.ext3 = (float)sqrt(G[4] / det23);
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) g.HK[a * 3 + c] = (float)(k.H[a * 3 + c] / Kd[a]);
    g.c2 = (float)(pl->pw_support * pl->pw_support);
    const double dV = k.vol / ((double)k.K1 * k.K2 * k.K3);
    g.wpref = (float)(dV / pow(2.0 * PW_PI, 1.5));
    // the support of the widest atom: at most a few grid lengths per axis
    // (a Gaussian far wider than the cell would visit many images per point)
    const int nb = (k.n + PW_NT - 1) / PW_NT;
    hipLaunchKernelGGL(k_pw_sigma_max, dim3(nb), dim3(PW_NT), 0, pl->stream, k.n, pl->sig, pl->pw_smax);
    QEQ_TRY(qeq_check(hipGetLastError()));
    std::vector<double> smax((size_t)nb);
    QEQ_HIP(hipMemcpyAsync(smax.data(), pl->pw_smax, sizeof(double) * nb, hipMemcpyDeviceToHost, pl->stream));
    QEQ_HIP(hipStreamSynchronize(pl->stream));
    double sm = 0.0;
    for (double v : smax) sm = std::max(sm, v);
    const double R = pl->pw_support * sm;
    for (int a = 0; a < 3; ++a)
        if (R * sqrt(Gi[a * 4]) > 4.0 * Kd[a]) return QEQ_EPLAN;
    return QEQ_OK;
}

static int pw_interp_launch(qeq_plan* pl, const double* src, const int* done, bool fin, int nb) {
    const KParams& k = pl->kp;
    if (fin)
        hipLaunchKernelGGL(k_pw_interp<true>, dim3(nb), dim3(PW_NT), 0, pl->stream, k, pl->pw_geom, src, pl->frac,
                           pl->sig, pl->grid_r, pl->pw_y, pl->pw_f, done);
    else
        hipLaunchKernelGGL(k_pw_interp<false>, dim3(nb), dim3(PW_NT), 0, pl->stream, k, pl->pw_geom, src, pl->frac,
                           pl->sig, pl->grid_r, pl->pw_y, pl->pw_f, done);
    return qeq_check(hipGetLastError());
}

// y = A src into pw_y (sorted order); with fin also the forces into pw_f.
int launch_pw_rec(qeq_plan* pl, const double* src, const int* done, bool fin) {
    const KParams& k = pl->kp;
    const size_t sh = sizeof(float2) * ((size_t)k.K3 + (size_t)k.K3 * (k.TW / 2));
    const int nb = pw_blocks(k.n);
    const size_t nreal = (size_t)k.K1 * k.K2 * k.K3;   // a multiple of 4 (K_a % 4 == 0)
    hipLaunchKernelGGL(k_pw_zero, dim3((unsigned)((nreal / 4 + PW_NT - 1) / PW_NT)), dim3(PW_NT), 0, pl->stream,
                       (float4*)pl->grid_r, nreal / 4, done);
    hipLaunchKernelGGL(k_pw_spread, dim3(nb), dim3(PW_NT), 0, pl->stream, k, pl->pw_geom, src, pl->frac, pl->sig,
                       pl->grid_r, done);
    if (sh > 65536)
        QEQ_HIP(hipFuncSetAttribute((const void*)k_pw_r2c, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));
    hipLaunchKernelGGL(k_pw_r2c, dim3(k.K1 * k.ntile), dim3(PW_NT), sh, pl->stream, k, pl->axes.ax[2],
                       pl->grid_r, pl->grid_c, done);
    QEQ_TRY(qeq_check(hipGetLastError()));
    QEQ_TRY(launch_mesh_from_spectrum(pl, done));
    return pw_interp_launch(pl, src, done, fin, nb);
}

int launch_pw_forces_add(qeq_plan* pl) {
    const int n = pl->kp.n;
    hipLaunchKernelGGL(k_pw_add_forces, dim3(nblocks(3 * n)), dim3(QEQ_BLOCK), 0, pl->stream, n, pl->pw_f,
                       pl->fdst);
    return qeq_check(hipGetLastError());
}
