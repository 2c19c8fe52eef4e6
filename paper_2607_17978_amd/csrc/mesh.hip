// Reciprocal-space part of the matrix-vector product (paper, "Electrostatics
// Solvers", eq. matvec): B-spline charge spreading, 3-D real-to-complex FFT,
// multiplication by the Gaussian-screened Green's function, inverse FFT.
//
// Layouts in HBM:
//   real grid      R[g1][g2][g3]           (g3 contiguous)
//   half spectrum  C[m3][m1][m2]           (m2 contiguous, m3 = 0 .. K3/2)
// Passes (each one read and one write of the grid, all in LDS):
//   1. spread + R2C along axis 3  : block = (g1, tile of TW rows g2); atoms whose
//      spline support touches the tile are accumulated with LDS atomics, two
//      real rows are packed into one complex FFT, the half spectra are written
//      transposed so that m2 becomes contiguous.
//   2. C2C along axis 2 (rows contiguous), NR rows per block.
//   3. C2C along axis 1 (stride K2) on tiles of TW columns: forward FFT,
//      multiplication by G(m) computed on the fly, inverse FFT, in one pass.
//   4. inverse C2C along axis 2.
//   5. C2R along axis 3 back to R[g1][g2][g3].
#include <math.h>

#include "internal.h"

namespace {

#define MESH_FWD 1
#define MESH_GREEN 2
#define MESH_INV 4
#define MESH_ENERGY 8

__global__ __launch_bounds__(QEQ_FFT_THREADS) void k_spread_r2c(
    KParams k, FftAxis ax3, const double* __restrict__ src, const int* __restrict__ bin_start,
    const int* __restrict__ home, const float* __restrict__ wts, float2* __restrict__ C,
    const int* __restrict__ done) {
    if (done && *done) return;
    extern __shared__ float2 sm[];
    float2* tw = sm;
    float2* buf = sm + k.K3;
    __shared__ int seg_lo[2 * QEQ_MAXP], seg_off[2 * QEQ_MAXP + 1], seg_k1[2 * QEQ_MAXP];
    __shared__ int nseg;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int g1 = blockIdx.x / k.ntile;
    const int g20 = (blockIdx.x - g1 * k.ntile) * k.TW;
    const int ncl = k.TWlog2 - 1;
    const int ncol = k.TW >> 1;
    const int K1 = k.K1, K2 = k.K2, K3 = k.K3, p = k.p;

    for (int t = tid; t < K3; t += nthr) tw[t] = ax3.tw[t];
    for (int t = tid; t < K3 * ncol; t += nthr) buf[t] = make_float2(0.f, 0.f);
    if (tid == 0) {
        int ns = 0, off = 0;
        const int span = k.TW + p - 1;   // homes g20 .. g20 + span - 1 reach this tile
        for (int k1 = 0; k1 < p; ++k1) {
            int h1 = g1 + k1;
            if (h1 >= K1) h1 -= K1;
            int lo = g20, hi = g20 + span;
            int b0 = h1 * K2;
            int a1 = lo, e1 = hi < K2 ? hi : K2;
            seg_lo[ns] = bin_start[b0 + a1];
            seg_k1[ns] = k1;
            seg_off[ns] = off;
            off += bin_start[b0 + e1] - bin_start[b0 + a1];
            ++ns;
            if (hi > K2) {
                seg_lo[ns] = bin_start[b0];
                seg_k1[ns] = k1;
                seg_off[ns] = off;
                off += bin_start[b0 + (hi - K2)] - bin_start[b0];
                ++ns;
            }
        }
        seg_off[ns] = off;
        nseg = ns;
    }
    __syncthreads();
    const int pp = p * p;
    const int total = seg_off[nseg] * pp;
    for (int item = tid; item < total; item += nthr) {
        int cidx = item / pp;
        int rem = item - cidx * pp;
        int k2 = rem / p;
        int k3 = rem - k2 * p;
        int sg = 0;
        while (cidx >= seg_off[sg + 1]) ++sg;
        int a = seg_lo[sg] + (cidx - seg_off[sg]);
        int k1 = seg_k1[sg];
        int h2 = home[4 * a + 1], h3 = home[4 * a + 2];
        int r = h2 - k2 - g20;
        if (r < 0) r += K2;
        if (r >= k.TW) continue;
        const float* w = wts + (size_t)a * 3 * QEQ_MAXP;
        float v = (float)src[a] * w[k1] * w[QEQ_MAXP + k2] * w[2 * QEQ_MAXP + k3];
        int g3 = h3 - k3;
        if (g3 < 0) g3 += K3;
        float* dst = reinterpret_cast<float*>(&buf[g3 * ncol + (r >> 1)]) + (r & 1);
        atomicAdd(dst, v);
    }
    __syncthreads();
    fft_lds(buf, ax3, ncl, tw, false, tid, nthr);
    // unpack the two real rows of each complex column and write the half spectra
    for (int t = tid; t < k.K3h * k.TW; t += nthr) {
        int r = t & (k.TW - 1);
        int m = t >> k.TWlog2;
        int pr = r >> 1;
        float2 Z = buf[m * ncol + pr];
        float2 Zc = buf[(m == 0 ? 0 : K3 - m) * ncol + pr];
        Zc.y = -Zc.y;
        float2 X;
        if ((r & 1) == 0) {
            X = make_float2(0.5f * (Z.x + Zc.x), 0.5f * (Z.y + Zc.y));
        } else {
            float2 d = csub(Z, Zc);
            X = make_float2(0.5f * d.y, -0.5f * d.x);
        }
        C[((size_t)m * K1 + g1) * K2 + g20 + r] = X;
    }
}

__global__ __launch_bounds__(QEQ_FFT_THREADS) void k_fft_rows(KParams k, FftAxis ax2,
                                                             float2* __restrict__ C, int nrows, int inv,
                                                             const int* __restrict__ done) {
    if (done && *done) return;
    extern __shared__ float2 sm[];
    float2* tw = sm;
    float2* buf = sm + k.K2;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int K2 = k.K2, NR = k.NR;
    const int row0 = blockIdx.x * NR;
    for (int t = tid; t < K2; t += nthr) tw[t] = ax2.tw[t];
    for (int t = tid; t < NR * K2; t += nthr) {
        int row = t / K2;
        int kk = t - row * K2;
        buf[kk * NR + row] = (row0 + row < nrows) ? C[(size_t)(row0 + row) * K2 + kk] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    fft_lds(buf, ax2, k.NRlog2, tw, inv != 0, tid, nthr);
    for (int t = tid; t < NR * K2; t += nthr) {
        int row = t / K2;
        int kk = t - row * K2;
        if (row0 + row < nrows) C[(size_t)(row0 + row) * K2 + kk] = buf[kk * NR + row];
    }
}

// Reciprocal kernel of the split (SI "Ewald Summation" Gaussian filter with the
// eq. matvec Poisson kernel 4 pi / k^2), times the B-spline moduli |b_a|^2:
//   G(m) = (4 pi / V) exp(-eta^2 k^2 / 2) / k^2 |b_1(m_1)|^2 |b_2(m_2)|^2 |b_3(m_3)|^2,
// k = 2 pi H^{-1} m; G = 0 at m = 0 and on the Nyquist planes (where the
// half-spectrum symmetry of a triclinic cell is ambiguous; the Gaussian there
// is below 1e-14 for grids at the supported spacings).
__device__ __forceinline__ float green_value(const KParams& k, int m1, int m2, int m3,
                                             const float* __restrict__ b1, const float* __restrict__ b2,
                                             const float* __restrict__ b3) {
    if ((m1 | m2 | m3) == 0) return 0.f;
    if (2 * m1 == k.K1 || 2 * m2 == k.K2 || 2 * m3 == k.K3) return 0.f;
    double x1 = m1 <= k.K1 / 2 ? m1 : m1 - k.K1;
    double x2 = m2 <= k.K2 / 2 ? m2 : m2 - k.K2;
    double x3 = m3;
    double q = k.M[0] * x1 * x1 + k.M[1] * x2 * x2 + k.M[2] * x3 * x3 +
               2.0 * (k.M[3] * x1 * x2 + k.M[4] * x1 * x3 + k.M[5] * x2 * x3);
    double k2 = 39.478417604357434475 * q;   // (2 pi)^2
    double g = k.green_pref * exp(-0.5 * k.eta * k.eta * k2) / k2;
    return (float)g * b1[m1] * b2[m2] * b3[m3];
}

__global__ __launch_bounds__(QEQ_FFT_THREADS) void k_fft_cols(
    KParams k, FftAxis ax1, float2* __restrict__ C, const float* __restrict__ b1,
    const float* __restrict__ b2, const float* __restrict__ b3, int mode, double* __restrict__ epart,
    const int* __restrict__ done) {
    if (done && *done) return;
    extern __shared__ float2 sm[];
    float2* tw = sm;
    float2* buf = sm + k.K1;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int K1 = k.K1, K2 = k.K2, TW = k.TW;
    const int m3 = blockIdx.x / k.ntile;
    const int g20 = (blockIdx.x - m3 * k.ntile) * TW;
    for (int t = tid; t < K1; t += nthr) tw[t] = ax1.tw[t];
    float2* base = C + (size_t)m3 * K1 * K2 + g20;
    for (int t = tid; t < K1 * TW; t += nthr) {
        int c = t & (TW - 1), g1 = t >> k.TWlog2;
        buf[t] = base[(size_t)g1 * K2 + c];
    }
    __syncthreads();
    if (mode & MESH_FWD) fft_lds(buf, ax1, k.TWlog2, tw, false, tid, nthr);
    if (mode & MESH_GREEN) {
        double e = 0.0;
        const float mult = (m3 == 0) ? 1.f : 2.f;
        for (int t = tid; t < K1 * TW; t += nthr) {
            int c = t & (TW - 1), m1 = t >> k.TWlog2;
            float g = green_value(k, m1, g20 + c, m3, b1, b2, b3);
            float2 x = buf[t];
            if (mode & MESH_ENERGY) e += (double)(g * mult * (x.x * x.x + x.y * x.y));
            buf[t] = make_float2(x.x * g, x.y * g);
        }
        if (mode & MESH_ENERGY) {
            double v[1] = {e};
            block_sum<1>(v);
            if (tid == 0) epart[blockIdx.x] = v[0];
        }
        __syncthreads();
    }
    if (mode & MESH_INV) fft_lds(buf, ax1, k.TWlog2, tw, true, tid, nthr);
    for (int t = tid; t < K1 * TW; t += nthr) {
        int c = t & (TW - 1), g1 = t >> k.TWlog2;
        base[(size_t)g1 * K2 + c] = buf[t];
    }
}

__global__ __launch_bounds__(QEQ_FFT_THREADS) void k_c2r(KParams k, FftAxis ax3,
                                                        const float2* __restrict__ C, float* __restrict__ R,
                                                        const int* __restrict__ done) {
    if (done && *done) return;
    extern __shared__ float2 sm[];
    const int K1 = k.K1, K2 = k.K2, K3 = k.K3, TW = k.TW;
    const int ncol = TW >> 1, ncl = k.TWlog2 - 1;
    float2* tw = sm;
    float2* X = sm + K3;
    float2* Z = X + k.K3h * TW;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int g1 = blockIdx.x / k.ntile;
    const int g20 = (blockIdx.x - g1 * k.ntile) * TW;
    for (int t = tid; t < K3; t += nthr) tw[t] = ax3.tw[t];
    for (int t = tid; t < k.K3h * TW; t += nthr) {
        int r = t & (TW - 1), m = t >> k.TWlog2;
        X[t] = C[((size_t)m * K1 + g1) * K2 + g20 + r];
    }
    __syncthreads();
    // Z = X_even + i X_odd over the full axis (Hermitian extension)
    for (int t = tid; t < K3 * ncol; t += nthr) {
        int pr = t & (ncol - 1), m = t >> ncl;
        float2 xa, xb;
        if (2 * m <= K3) {
            xa = X[m * TW + 2 * pr];
            xb = X[m * TW + 2 * pr + 1];
        } else {
            xa = X[(K3 - m) * TW + 2 * pr];
            xb = X[(K3 - m) * TW + 2 * pr + 1];
            xa.y = -xa.y;
            xb.y = -xb.y;
        }
        Z[t] = make_float2(xa.x - xb.y, xa.y + xb.x);
    }
    __syncthreads();
    fft_lds(Z, ax3, ncl, tw, true, tid, nthr);
    for (int r = 0; r < TW; ++r) {
        float* dst = R + ((size_t)g1 * K2 + g20 + r) * K3;
        const float* zs = reinterpret_cast<const float*>(Z) + (r >> 1) * 2 + (r & 1);
        for (int g3 = tid; g3 < K3; g3 += nthr) dst[g3] = zs[g3 * 2 * ncol];
    }
}

__global__ void k_write_green(KParams k, float2* __restrict__ C, const float* __restrict__ b1,
                              const float* __restrict__ b2, const float* __restrict__ b3) {
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t total = (size_t)k.K3h * k.K1 * k.K2;
    if (t >= total) return;
    int m2 = (int)(t % k.K2);
    int m1 = (int)((t / k.K2) % k.K1);
    int m3 = (int)(t / ((size_t)k.K2 * k.K1));
    C[t] = make_float2(green_value(k, m1, m2, m3, b1, b2, b3), 0.f);
}

size_t smem_spread(const KParams& k) { return sizeof(float2) * ((size_t)k.K3 + (size_t)k.K3 * (k.TW / 2)); }
size_t smem_rows(const KParams& k) { return sizeof(float2) * ((size_t)k.K2 + (size_t)k.K2 * k.NR); }
size_t smem_cols(const KParams& k) { return sizeof(float2) * ((size_t)k.K1 + (size_t)k.K1 * k.TW); }
size_t smem_c2r(const KParams& k) {
    return sizeof(float2) * ((size_t)k.K3 + (size_t)k.K3h * k.TW + (size_t)k.K3 * (k.TW / 2));
}

int rows_pass(qeq_plan* pl, int inv, const int* done) {
    const KParams& k = pl->kp;
    ProfScope ps(pl, inv ? PK_ROWS_INV : PK_ROWS_FWD);
    int nrows = k.K3h * k.K1;
    hipLaunchKernelGGL(k_fft_rows, dim3((nrows + k.NR - 1) / k.NR), dim3(QEQ_FFT_THREADS),
                       smem_rows(k), pl->stream, k, pl->axes.ax[1], pl->grid_c, nrows, inv, done);
    return qeq_check(hipGetLastError());
}

int cols_pass(qeq_plan* pl, int mode, double* epart, const int* done) {
    const KParams& k = pl->kp;
    ProfScope ps(pl, PK_COLS_GREEN);
    hipLaunchKernelGGL(k_fft_cols, dim3(k.K3h * k.ntile), dim3(QEQ_FFT_THREADS), smem_cols(k),
                       pl->stream, k, pl->axes.ax[0], pl->grid_c, pl->bmod[0], pl->bmod[1],
                       pl->bmod[2], mode, epart, done);
    return qeq_check(hipGetLastError());
}

int c2r_pass(qeq_plan* pl, const int* done) {
    const KParams& k = pl->kp;
    ProfScope ps(pl, PK_C2R);
    hipLaunchKernelGGL(k_c2r, dim3(k.K1 * k.ntile), dim3(QEQ_FFT_THREADS), smem_c2r(k), pl->stream,
                       k, pl->axes.ax[2], pl->grid_c, pl->grid_r, done);
    return qeq_check(hipGetLastError());
}

}  // namespace

size_t qeq_mesh_max_smem(const KParams& k) {
    size_t a = smem_spread(k), b = smem_rows(k), c = smem_cols(k), d = smem_c2r(k);
    size_t m = a > b ? a : b;
    m = m > c ? m : c;
    return m > d ? m : d;
}

int launch_mesh_potential(qeq_plan* pl, const double* src, const int* done) {
    const KParams& k = pl->kp;
    {
        ProfScope ps(pl, PK_SPREAD_R2C);
        hipLaunchKernelGGL(k_spread_r2c, dim3(k.K1 * k.ntile), dim3(QEQ_FFT_THREADS), smem_spread(k),
                       pl->stream, k, pl->axes.ax[2], src, pl->bin_start, pl->home, pl->wts,
                       pl->grid_c, done);
    }
    QEQ_HIP(hipGetLastError());
    QEQ_TRY(rows_pass(pl, 0, done));
    QEQ_TRY(cols_pass(pl, MESH_FWD | MESH_GREEN | MESH_INV, nullptr, done));
    QEQ_TRY(rows_pass(pl, 1, done));
    return c2r_pass(pl, done);
}

int launch_mesh_inverse(qeq_plan* pl) {
    QEQ_TRY(cols_pass(pl, MESH_INV, nullptr, nullptr));
    QEQ_TRY(rows_pass(pl, 1, nullptr));
    return c2r_pass(pl, nullptr);
}

int launch_write_green(qeq_plan* pl) {
    const KParams& k = pl->kp;
    size_t total = (size_t)k.K3h * k.K1 * k.K2;
    hipLaunchKernelGGL(k_write_green, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, pl->stream,
                       k, pl->grid_c, pl->bmod[0], pl->bmod[1], pl->bmod[2]);
    return qeq_check(hipGetLastError());
}
