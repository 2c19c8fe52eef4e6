// Reciprocal-space part of the matrix-vector product (paper, "Electrostatics
// Solvers", eq. matvec): B-spline charge spreading, 3-D real-to-complex FFT,
// multiplication by the Gaussian-screened Green's function, inverse FFT.
//
// Layouts in HBM:
//   real grid      R[g1][g2][g3]           (g3 contiguous)
//   half spectrum  C[m3][m1][m2]           (m2 contiguous, m3 = 0 .. K3/2)
// Passes (each one read and one write of the grid, transforms in LDS):
//   1. spread + R2C along axis 3  : block = (g1, tile of TW rows g2).  The
//      atoms whose spline support reaches the tile are held in registers (one
//      per thread), their weights accumulated into the tile in 32-bit fixed
//      point with integer LDS atomics (order-independent sums; FP32 LDS
//      atomics run at a fraction of the integer rate on gfx950), converted
//      to FP32, two real rows packed into one complex FFT and the half
//      spectra written transposed so that m2 becomes contiguous.
//   2. C2C along axis 2 (rows contiguous), NR rows per block.
//   3. C2C along axis 1 (stride K2) on tiles of TW columns: forward FFT,
//      multiplication by G(m) computed on the fly, inverse FFT, in one pass.
//   4. inverse C2C along axis 2.
//   5. C2R along axis 3 back to R[g1][g2][g3].
// Every pass is a template on its axis length (and tile width, spline order):
// the common lengths get fully compile-time transforms, any other supported
// length runs the same kernel with runtime sizes (template value 0).
#include <math.h>

#include "internal.h"

namespace {

#define MESH_FWD 1
#define MESH_GREEN 2
#define MESH_INV 4
#define MESH_ENERGY 8


constexpr int NT = QEQ_FFT_THREADS;

__device__ __forceinline__ int ilog2_dev(int x) { return 31 - __clz(x); }


// ------------------------------------------------------------------ pass 1
template <int KC, int TWC, int PC>
__global__ __launch_bounds__(NT) void k_spread_r2c(KParams k, FftAxis ax3, const double* __restrict__ src,
                                                  const int* __restrict__ bin_start,
                                                  const int* __restrict__ home,
                                                  const float* __restrict__ wts, float2* __restrict__ C,
                                                  const int* __restrict__ done) {
    extern __shared__ float2 sm[];
    const int K3 = KC ? KC : k.K3;
    const int TW = TWC ? TWC : k.TWS;
    const int p = PC ? PC : k.p;
    const int ncol = TW >> 1;
    // LDS: twiddles | accumulator acc[g3][row] (int32; the FFT buffer
    // buf[g3][pr] (complex, two rows per element) takes its place once
    // converted)
    float2* tw = sm;
    int* acc = reinterpret_cast<int*>(sm + K3);
    float2* buf = sm + K3;
    __shared__ int seg_lo[2 * QEQ_MAXP], seg_off[2 * QEQ_MAXP + 1], seg_k1[2 * QEQ_MAXP];
    __shared__ int seg_len[2 * QEQ_MAXP];
    __shared__ float sh_scale;
    const int tid = threadIdx.x;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int g1 = blk / k.ntile_s;
    const int g20 = (blk - g1 * k.ntile_s) * TW;
    const int K1 = k.K1, K2 = k.K2;

    // The twiddles and the candidate bin bounds are requested before the
    // converged flag is examined, so the three loads share one round trip.
    // Candidate segments: for each k1, homes h1 = g1 + k1 and h2 in
    // [g20, g20 + TW + p - 1) (two pieces when the h2 range wraps); lanes
    // k1 < p fetch their bounds.
    constexpr bool TW1 = KC > 0;
    constexpr int PT = KC > 0 ? (KC + NT - 1) / NT : 1;
    float2 twv[PT];
#pragma unroll
    for (int u = 0; u < PT; ++u)
        if (TW1 && tid + u * NT < K3) twv[u] = ax3.tw[tid + u * NT];
    int lo0 = 0, len0 = 0, lo1 = 0, len1 = 0;
    if (tid < p) {
        int h1 = g1 + tid;
        if (h1 >= K1) h1 -= K1;
        const int b0 = h1 * K2;
        const int hi = g20 + TW + p - 1;
        const int e1 = hi < K2 ? hi : K2;
        lo0 = bin_start[b0 + g20];
        len0 = bin_start[b0 + e1];
        if (hi > K2) {
            lo1 = bin_start[b0];
            len1 = bin_start[b0 + (hi - K2)];
        }
    }
    if (done && *done) return;
    if (TW1) {
#pragma unroll
        for (int u = 0; u < PT; ++u)
            if (tid + u * NT < K3) tw[tid + u * NT] = twv[u];
    } else {
        for (int t = tid; t < K3; t += NT) tw[t] = ax3.tw[t];
    }
    for (int t = tid; t < K3 * TW; t += NT) acc[t] = 0;
    if (tid < p) {
        seg_lo[2 * tid] = lo0;
        seg_len[2 * tid] = len0 - lo0;
        seg_lo[2 * tid + 1] = lo1;
        seg_len[2 * tid + 1] = len1 - lo1;
        seg_k1[2 * tid] = tid;
        seg_k1[2 * tid + 1] = tid;
    }
    __syncthreads();
    if (tid == 0) {
        int off = 0;
        for (int sg = 0; sg < 2 * p; ++sg) {
            seg_off[sg] = off;
            off += seg_len[sg];
        }
        seg_off[2 * p] = off;
    }
    __syncthreads();
    const int ncand = seg_off[2 * p];
    // Candidate c of a round is held by thread c in registers: its
    // source value times the axis-1 weight, the axis-2 and axis-3 weights and
    // its home indices (no LDS staging, so more blocks fit per CU).
    constexpr int PM = PC ? PC : QEQ_MAXP;
    float a0 = 0.f, w2[PM], w3[PM];
    int h2 = 0, h3 = 0;
    double abound = 0.0;
    auto seg_of = [&](int cidx) {
        // last segment starting at or before cidx (empty segments share their
        // start with the next one and are passed over); independent LDS reads
        int sg = 0;
#pragma unroll
        for (int s2 = 1; s2 < 2 * PM; ++s2) {
            if (!PC && s2 >= 2 * p) break;
            sg += cidx >= seg_off[s2] ? 1 : 0;
        }
        return sg;
    };
    auto load_cand = [&](int cidx) {
        const int sg = seg_of(cidx);
        const int a = seg_lo[sg] + (cidx - seg_off[sg]);
        const float* w = wts + (size_t)a * 3 * QEQ_MAXP;
        const double sv = src[a];
        const float w1 = w[seg_k1[sg]];
        a0 = (float)sv * w1;
        float m2 = 0.f, m3 = 0.f;
#pragma unroll
        for (int kk = 0; kk < PM; ++kk) {
            if (!PC && kk >= p) break;
            w2[kk] = w[QEQ_MAXP + kk];
            w3[kk] = w[2 * QEQ_MAXP + kk];
            m2 = fmaxf(m2, w2[kk]);
            m3 = fmaxf(m3, w3[kk]);
        }
        abound = fabs(sv) * (double)w1 * (double)m2 * (double)m3;
        h2 = home[4 * a + 1];
        h3 = home[4 * a + 2];
    };
    // Fixed-point scale: every grid value of the tile is a sum over the
    // candidates of one term each, src w1(k1) w2(k2) w3(k3), so |value| <=
    // S = sum over candidates of |src| w1 max(w2) max(w3); with scale =
    // 2^(30 - e), S < 2^e, every scaled term and partial sum (rounding of
    // each term included) stays below 2^31 in magnitude.  The step 2^(e-30)
    // is at most 2^-29 S: with the weight maxima in S, about the rounding
    // of the FP32 transforms that follow.  One round: S from the registers;
    // more rounds: a pass over the candidates first.
    const bool one_round = ncand <= NT;
    {
        double v[1] = {0.0};
        if (one_round) {
            if (tid < ncand) {
                load_cand(tid);
                v[0] = abound;
            }
        } else {
            for (int cidx = tid; cidx < ncand; cidx += NT) {
                load_cand(cidx);
                v[0] += abound;
            }
        }
        block_sum<1>(v);
        if (tid == 0) {
            int e = 0;
            (void)frexp(v[0] > 0.0 ? v[0] : 1.0, &e);   // v < 2^e
            sh_scale = ldexpf(1.0f, max(-126, min(126, 30 - e)));
        }
        __syncthreads();
    }
    const float scale = sh_scale;
    // A term t (|t| < 2^31) becomes an integer by one FP64 fused multiply-add
    // with 1.5 * 2^52: the sum lies in [2^52, 2^53), where the spacing of
    // doubles is 1, so it is t rounded to the nearest integer plus 2^52 + 2^51,
    // and the low word of its bit pattern (that of 1.5 * 2^52 is zero) is the
    // two's-complement integer.
    constexpr double RND = 6755399441055744.0;   // 1.5 * 2^52
    for (int base = 0; base < ncand; base += NT) {
        const int cidx = base + tid;
        if (cidx < ncand) {
            if (!one_round) load_cand(cidx);
            const double as = (double)(a0 * scale);
            double w3d[PM];
            int col[PM];
#pragma unroll
            for (int k3 = 0; k3 < PM; ++k3) {
                if (!PC && k3 >= p) break;
                w3d[k3] = (double)w3[k3];
                int g3 = h3 - k3;
                if (g3 < 0) g3 += K3;
                col[k3] = g3 * TW;
            }
#pragma unroll
            for (int k2 = 0; k2 < PM; ++k2) {
                if (!PC && k2 >= p) break;
                // row of grid point h2 - k2 inside this tile; a tile narrower
                // than p - 1 rows also sees candidates whose point lies before it
                int r = h2 - k2 - g20;
                if (r < 0) r += K2;
                if (r < 0 || r >= TW) continue;
                const double a1 = as * (double)w2[k2];   // exact: two 24-bit significands
#pragma unroll
                for (int k3 = 0; k3 < PM; ++k3) {
                    if (!PC && k3 >= p) break;
                    const int t = (int)(unsigned)__double_as_longlong(fma(a1, w3d[k3], RND));
                    atomicAdd(acc + col[k3] + r, t);
                }
            }
        }
    }
    __syncthreads();
    // fixed point -> FP32, packed two real rows per complex column, then the
    // axis-3 transform
    const float inv = 1.0f / scale;
    if constexpr (KC > 0 && TWC > 0) {
        // the conversion happens inside the first radix stage: each item
        // reads the fixed-point values of its R0 inputs into registers, and
        // after the barrier the stage's outputs overwrite the accumulator
        constexpr int NCS = TWC / 2;
        constexpr int R0 = ct_radix_at(KC, 0, NCS, NT), PER0 = KC / R0;
        constexpr int ITEMS = PER0 * NCS, IT0 = (ITEMS + NT - 1) / NT;
        float2 v[IT0][R0];
#pragma unroll
        for (int it = 0; it < IT0; ++it) {
            const int item = tid + it * NT;
            if (ITEMS % NT == 0 || item < ITEMS) {
                const int c = item % NCS, j = item / NCS;
#pragma unroll
                for (int r = 0; r < R0; ++r) {
                    const int2 a = *reinterpret_cast<const int2*>(acc + (j + r * PER0) * TWC + 2 * c);
                    v[it][r] = make_float2((float)a.x * inv, (float)a.y * inv);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < IT0; ++it) {
            const int item = tid + it * NT;
            if (ITEMS % NT == 0 || item < ITEMS) {
                const int c = item % NCS, j = item / NCS;
                dft<R0>(v[it], false);
#pragma unroll
                for (int r = 0; r < R0; ++r) buf[(j * R0 + r) * NCS + c] = v[it][r];
            }
        }
        __syncthreads();
        fft_ct<KC, NCS, NCS, NT, false, 1, R0>(buf, tw, tid);
    } else {
        // runtime sizes: convert through registers one chunk of NT at a time
        for (int e0 = 0; e0 < K3 * ncol; e0 += NT) {
            const int e = e0 + tid;
            float2 v = make_float2(0.f, 0.f);
            if (e < K3 * ncol) {
                const int g3 = e / ncol, pr = e - g3 * ncol;
                v = make_float2((float)acc[g3 * TW + 2 * pr] * inv, (float)acc[g3 * TW + 2 * pr + 1] * inv);
            }
            __syncthreads();
            if (e < K3 * ncol) buf[e] = v;
            __syncthreads();
        }
        __syncthreads();
        fft_lds(buf, ax3, ilog2_dev(ncol), tw, false, tid, NT);
    }
    // unpack the two real rows of each complex column and write the half spectra
    const int K3h = K3 / 2 + 1;
    if constexpr (KC > 0 && TWC > 0) {
        // compile-time tiles: every LDS read of the thread first, then the
        // unpacking (both rows' formulas, selected) and the stores
        constexpr int NW = (KC / 2 + 1) * TWC, PW = (NW + NT - 1) / NT, NCS = TWC / 2;
        float2 zv[PW], zc[PW];
#pragma unroll
        for (int u = 0; u < PW; ++u) {
            const int t = tid + u * NT;
            if (NW % NT == 0 || t < NW) {
                const int m = t / TWC, pr = (t - m * TWC) >> 1;
                zv[u] = buf[m * NCS + pr];
                zc[u] = buf[(m == 0 ? 0 : KC - m) * NCS + pr];
            }
        }
#pragma unroll
        for (int u = 0; u < PW; ++u) {
            const int t = tid + u * NT;
            if (NW % NT == 0 || t < NW) {
                const int m = t / TWC, r = t - m * TWC;
                const float2 Z = zv[u], Zc = make_float2(zc[u].x, -zc[u].y);
                const float2 ev = make_float2(0.5f * (Z.x + Zc.x), 0.5f * (Z.y + Zc.y));
                const float2 d = csub(Z, Zc);
                const float2 od = make_float2(0.5f * d.y, -0.5f * d.x);
                C[((size_t)m * K1 + g1) * K2 + g20 + r] = (r & 1) ? od : ev;
            }
        }
        return;
    }
    const int twl = ilog2_dev(TW);
    for (int t = tid; t < K3h * TW; t += NT) {
        // compile-time tiles may have any even width (division by a constant)
        const int m = TWC ? t / TWC : t >> twl;
        const int r = t - m * TW;
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

// ------------------------------------------------------------------ passes 2 / 4
// LDS layout [k][row] with row stride NR + 1 (odd) for the compile-time path,
// which keeps the transposing loads and stores free of bank conflicts.
template <int KC, int NRC, bool INV>
__global__ __launch_bounds__(NT) void k_fft_rows(KParams k, FftAxis ax2, float2* __restrict__ C, int nrows,
                                                const int* __restrict__ done) {
    if (done && *done) return;
    extern __shared__ float2 sm[];
    const int K2 = KC ? KC : k.K2;
    const int NR = NRC ? NRC : k.NR;
    const int KS = NRC ? NRC + 1 : NR;
    float2* tw = sm;
    float2* buf = sm + K2;
    const int tid = threadIdx.x;
    const int row0 = blockIdx.x * NR;
    auto ld_tw = [&](int t) { return ax2.tw[t]; };
    auto st_tw = [&](int t, float2 v) { tw[t] = v; };
    auto ld = [&](int t) {
        const int row = t / K2, kk = t - row * K2;
        return (row0 + row < nrows) ? C[(size_t)(row0 + row) * K2 + kk] : make_float2(0.f, 0.f);
    };
    auto st = [&](int t, float2 v) {
        const int row = t / K2, kk = t - row * K2;
        buf[kk * KS + row] = v;
    };
    if constexpr (KC > 0 && NRC > 0) {
        stage2_ct<KC, NRC * KC, NT, float2>(tid, ld_tw, st_tw, ld, st);
    } else {
        stage_rt<4, float2>(K2, tid, NT, ld_tw, st_tw);
        stage_rt<4, float2>(NR * K2, tid, NT, ld, st);
    }
    __syncthreads();
    if constexpr (KC > 0 && NRC > 0)
        fft_ct<KC, NRC, NRC + 1, NT, INV>(buf, tw, tid);
    else
        fft_lds(buf, ax2, k.NRlog2, tw, INV, tid, NT);
    auto ld_out = [&](int t) {
        const int row = t / K2, kk = t - row * K2;
        return buf[kk * KS + row];
    };
    auto st_out = [&](int t, float2 v) {
        const int row = t / K2, kk = t - row * K2;
        if (row0 + row < nrows) C[(size_t)(row0 + row) * K2 + kk] = v;
    };
    if constexpr (KC > 0 && NRC > 0)
        stage_ct<NRC * KC, NT, float2>(tid, ld_out, st_out);   // LDS reads first, then the stores
    else
        stage_rt<4, float2>(NR * K2, tid, NT, ld_out, st_out);
}

// Reciprocal kernel of the split (SI "Ewald Summation" Gaussian filter with the
// eq. matvec Poisson kernel 4 pi / k^2), times the B-spline moduli |b_a|^2:
//   G(m) = (4 pi / V) exp(-eta^2 k^2 / 2) / k^2 |b_1(m_1)|^2 |b_2(m_2)|^2 |b_3(m_3)|^2,
// k = 2 pi H^{-1} m; G = 0 at m = 0 and on the Nyquist planes (where the
// half-spectrum symmetry of a triclinic cell is ambiguous; the Gaussian there
// is below 1e-14 for grids at the supported spacings).  Evaluated in FP32: it
// multiplies an FP32 spectrum, and FP32 exp / divide keep its relative error
// at a few ulp.
__device__ __forceinline__ float green_core(const KParams& k, int m1, int m2, int m3) {
    if ((m1 | m2 | m3) == 0) return 0.f;
    if (2 * m1 == k.K1 || 2 * m2 == k.K2 || 2 * m3 == k.K3) return 0.f;
    const float x1 = (float)(m1 <= k.K1 / 2 ? m1 : m1 - k.K1);
    const float x2 = (float)(m2 <= k.K2 / 2 ? m2 : m2 - k.K2);
    const float x3 = (float)m3;
    const float q = (float)k.M[0] * x1 * x1 + (float)k.M[1] * x2 * x2 + (float)k.M[2] * x3 * x3 +
                    2.0f * ((float)k.M[3] * x1 * x2 + (float)k.M[4] * x1 * x3 + (float)k.M[5] * x2 * x3);
    const float k2 = 39.478417604357434475f * q;   // (2 pi)^2
    const float eta = (float)k.eta_green;
    return (float)k.green_pref * expf(-0.5f * eta * eta * k2) / k2;
}

__device__ __forceinline__ float green_value(const KParams& k, int m1, int m2, int m3,
                                             const float* __restrict__ b1, const float* __restrict__ b2,
                                             const float* __restrict__ b3) {
    const float g = green_core(k, m1, m2, m3);
    return g * b1[m1] * b2[m2] * b3[m3];
}

// ------------------------------------------------------------------ pass 3
template <int KC, int TWC>
__global__ __launch_bounds__(NT) void k_fft_cols(KParams k, FftAxis ax1, float2* __restrict__ C,
                                                const float* __restrict__ b1, const float* __restrict__ b2,
                                                const float* __restrict__ b3, int mode,
                                                double* __restrict__ epart, const int* __restrict__ done) {
    if (done && *done) return;
    extern __shared__ float2 sm[];
    const int K1 = KC ? KC : k.K1;
    const int TW = TWC ? TWC : k.TW;
    const int twl = ilog2_dev(TW);
    float2* tw = sm;
    float2* buf = sm + K1;
    const int tid = threadIdx.x;
    const int K2 = k.K2;
    const int m3 = blockIdx.x / k.ntile;
    const int g20 = (blockIdx.x - m3 * k.ntile) * TW;
    float2* base = C + (size_t)m3 * K1 * K2 + g20;
    constexpr bool CT = KC > 0 && TWC > 0;
    if constexpr (CT) {
        if ((mode & (MESH_FWD | MESH_GREEN | MESH_INV)) == (MESH_FWD | MESH_GREEN | MESH_INV)) {
            // The full product pass with the global-memory traffic folded into
            // the transforms: the forward transform's first radix stage reads
            // its inputs from HBM, the Green's function multiplies the inverse
            // transform's first-stage inputs as they are read, and the
            // inverse transform's last stage stores straight to HBM; each
            // saves an LDS pass and a barrier.  Every item of every stage
            // keeps the thread's column c = tid mod TW (NT is a multiple of
            // TW), so the Green's function's m2 is fixed per thread.
            constexpr int R0 = ct_radix_at(KC, 0, TWC, NT), PER0 = KC / R0;
            constexpr int IT0 = (PER0 * TWC + NT - 1) / NT;
            constexpr int NST = ct_nstages(KC, TWC, NT);
            static_assert(NST >= 2, "the first and the last stage are distinct");
            constexpr int RL = ct_radix_at(KC, NST - 1, TWC, NT), NSL = ct_span(KC, NST - 1, TWC, NT), PERL = KC / RL;
            constexpr int ITL = (PERL * TWC + NT - 1) / NT;
            constexpr int PT = (KC + NT - 1) / NT;
            const int c = tid & (TWC - 1);
            const int m2 = g20 + c;
            float2 twv[PT], v[IT0][R0];
            float bmv[IT0][R0];
            // twiddles, the tile and the moduli of the thread's elements, all
            // requested before any is used
#pragma unroll
            for (int u = 0; u < PT; ++u)
                if (tid + u * NT < KC) twv[u] = ax1.tw[tid + u * NT];
#pragma unroll
            for (int it = 0; it < IT0; ++it) {
                const int item = tid + it * NT;
                if ((PER0 * TWC) % NT == 0 || item < PER0 * TWC) {
                    const int j = item / TWC;
#pragma unroll
                    for (int r = 0; r < R0; ++r) {
                        const int g1 = j + r * PER0;
                        v[it][r] = base[(size_t)g1 * K2 + c];
                        bmv[it][r] = b1[g1];   // index of the same element after the transform
                    }
                }
            }
            const float bm23v = b2[m2] * b3[m3];
#pragma unroll
            for (int u = 0; u < PT; ++u)
                if (tid + u * NT < KC) tw[tid + u * NT] = twv[u];
            // forward transform: first stage from registers (no twiddles), the rest in LDS
#pragma unroll
            for (int it = 0; it < IT0; ++it) {
                const int item = tid + it * NT;
                if ((PER0 * TWC) % NT == 0 || item < PER0 * TWC) {
                    const int j = item / TWC;
                    dft<R0>(v[it], false);
#pragma unroll
                    for (int r = 0; r < R0; ++r) buf[(j * R0 + r) * TWC + c] = v[it][r];
                }
            }
            __syncthreads();
            fft_ct<KC, TWC, TWC, NT, false, 1, R0>(buf, tw, tid);
            // Green's function on the inverse transform's first-stage inputs
            // (the quadratic form k^2 / (2 pi)^2 = M11 x1^2 + l1 x1 + q23,
            // hardware exp2 and reciprocal)
            const float x2 = (float)(m2 <= k.K2 / 2 ? m2 : m2 - k.K2), x3 = (float)m3;
            const float M11 = (float)k.M[0];
            const float l1 = 2.0f * ((float)k.M[3] * x2 + (float)k.M[4] * x3);
            const float q23 = (float)k.M[1] * x2 * x2 + (float)k.M[2] * x3 * x3 + 2.0f * (float)k.M[5] * x2 * x3;
            const float eta = (float)k.eta_green;
            const float ce = -0.5f * eta * eta * 39.478417604357434475f * 1.4426950408889634f;
            const float pref = (float)k.green_pref / 39.478417604357434475f;
            const bool nyq23 = 2 * m2 == k.K2 || 2 * m3 == k.K3;
            const float mult = (m3 == 0) ? 1.f : 2.f;
            double e = 0.0;
#pragma unroll
            for (int it = 0; it < IT0; ++it) {
                const int item = tid + it * NT;
                if ((PER0 * TWC) % NT == 0 || item < PER0 * TWC) {
                    const int j = item / TWC;
#pragma unroll
                    for (int r = 0; r < R0; ++r) {
                        const int m1 = j + r * PER0;
                        const float x1 = (float)(m1 <= KC / 2 ? m1 : m1 - KC);
                        const float q = fmaf(fmaf(M11, x1, l1), x1, q23);
                        float g = pref * __builtin_amdgcn_exp2f(ce * q) * __builtin_amdgcn_rcpf(q) *
                                  (bmv[it][r] * bm23v);
                        if (nyq23 || 2 * m1 == KC || (m1 | m2 | m3) == 0) g = 0.f;
                        const float2 x = buf[m1 * TWC + c];
                        if (mode & MESH_ENERGY) e += (double)(g * mult * (x.x * x.x + x.y * x.y));
                        v[it][r] = make_float2(x.x * g, x.y * g);
                    }
                }
            }
            if (mode & MESH_ENERGY) {
                double ev[1] = {e};
                block_sum<1>(ev);
                if (tid == 0) epart[blockIdx.x] = ev[0];
            }
            __syncthreads();
#pragma unroll
            for (int it = 0; it < IT0; ++it) {
                const int item = tid + it * NT;
                if ((PER0 * TWC) % NT == 0 || item < PER0 * TWC) {
                    const int j = item / TWC;
                    dft<R0>(v[it], true);
#pragma unroll
                    for (int r = 0; r < R0; ++r) buf[(j * R0 + r) * TWC + c] = v[it][r];
                }
            }
            __syncthreads();
            fft_ct<KC, TWC, TWC, NT, true, 1, R0, 1, NST - 1>(buf, tw, tid);
            // last inverse stage: LDS to registers, twiddles, DFT, stores to HBM
            constexpr int STEPL = KC / (NSL * RL);
#pragma unroll
            for (int it = 0; it < ITL; ++it) {
                const int item = tid + it * NT;
                if ((PERL * TWC) % NT == 0 || item < PERL * TWC) {
                    const int j = item / TWC;
                    float2 u[RL];
#pragma unroll
                    for (int r = 0; r < RL; ++r) u[r] = buf[(j + r * PERL) * TWC + c];
                    const int kk = j % NSL;
#pragma unroll
                    for (int r = 1; r < RL; ++r) {
                        float2 w = tw[kk * r * STEPL];
                        w.y = -w.y;
                        u[r] = cmul(u[r], w);
                    }
                    dft<RL>(u, true);
                    const int bk = (j - kk) * RL + kk;
#pragma unroll
                    for (int r = 0; r < RL; ++r) base[(size_t)(bk + r * NSL) * K2 + c] = u[r];
                }
            }
            return;
        }
    }
    // compile-time tiles: the B-spline moduli of the Green's function are
    // loaded with the tile (a thread's column c = t mod TW is the same for all
    // its elements, since NT is a multiple of TW)
    constexpr int PER = CT ? (KC * TWC + NT - 1) / NT : 1;
    float bm1[PER];
    float bm23 = 0.f;
    if (CT && (mode & MESH_GREEN)) {
        bm23 = b2[g20 + (tid & (TW - 1))] * b3[m3];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int t = tid + u * NT;
            bm1[u] = (t < K1 * TW) ? b1[t >> twl] : 0.f;
        }
    }
    auto ld_tw = [&](int t) { return ax1.tw[t]; };
    auto st_tw = [&](int t, float2 v) { tw[t] = v; };
    auto ld = [&](int t) {
        const int c = t & (TW - 1), g1 = t >> twl;
        return base[(size_t)g1 * K2 + c];
    };
    auto st = [&](int t, float2 v) { buf[t] = v; };
    if constexpr (CT) {
        stage2_ct<KC, KC * TWC, NT, float2>(tid, ld_tw, st_tw, ld, st);
    } else {
        stage_rt<4, float2>(K1, tid, NT, ld_tw, st_tw);
        stage_rt<4, float2>(K1 * TW, tid, NT, ld, st);
    }
    __syncthreads();
    if (mode & MESH_FWD) {
        if constexpr (KC > 0 && TWC > 0)
            fft_ct<KC, TWC, TWC, NT, false>(buf, tw, tid);
        else
            fft_lds(buf, ax1, twl, tw, false, tid, NT);
    }
    if (mode & MESH_GREEN) {
        double e = 0.0;
        const float mult = (m3 == 0) ? 1.f : 2.f;
        if constexpr (CT) {
            // a thread's elements share m2 (its column) and m3 (the block's):
            // the quadratic form k^2 / (2 pi)^2 = M11 x1^2 + l1 x1 + q23 is two
            // FMAs per element, and the screened kernel uses the hardware
            // exponential and reciprocal (a few ulp, far below the FP32
            // spectrum's own rounding where G is not already negligible)
            const int m2 = g20 + (tid & (TW - 1));
            const float x2 = (float)(m2 <= k.K2 / 2 ? m2 : m2 - k.K2), x3 = (float)m3;
            const float M11 = (float)k.M[0];
            const float l1 = 2.0f * ((float)k.M[3] * x2 + (float)k.M[4] * x3);
            const float q23 = (float)k.M[1] * x2 * x2 + (float)k.M[2] * x3 * x3 + 2.0f * (float)k.M[5] * x2 * x3;
            const float eta = (float)k.eta_green;
            // exp(-eta^2 k^2 / 2) = 2^(ce q): ce = -eta^2 (2 pi)^2 log2(e) / 2
            const float ce = -0.5f * eta * eta * 39.478417604357434475f * 1.4426950408889634f;
            const float pref = (float)k.green_pref / 39.478417604357434475f;
            const bool nyq23 = 2 * m2 == k.K2 || 2 * m3 == k.K3;
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int t = tid + u * NT;
                if (t >= K1 * TW) break;
                const int m1 = t >> twl;
                const float x1 = (float)(m1 <= K1 / 2 ? m1 : m1 - K1);
                const float q = fmaf(fmaf(M11, x1, l1), x1, q23);
                float g = pref * __builtin_amdgcn_exp2f(ce * q) * __builtin_amdgcn_rcpf(q) * (bm1[u] * bm23);
                if (nyq23 || 2 * m1 == K1 || (m1 | m2 | m3) == 0) g = 0.f;
                const float2 x = buf[t];
                if (mode & MESH_ENERGY) e += (double)(g * mult * (x.x * x.x + x.y * x.y));
                buf[t] = make_float2(x.x * g, x.y * g);
            }
        } else {
            for (int t = tid; t < K1 * TW; t += NT) {
                const int c = t & (TW - 1), m1 = t >> twl;
                const float g = green_value(k, m1, g20 + c, m3, b1, b2, b3);
                const float2 x = buf[t];
                if (mode & MESH_ENERGY) e += (double)(g * mult * (x.x * x.x + x.y * x.y));
                buf[t] = make_float2(x.x * g, x.y * g);
            }
        }
        if (mode & MESH_ENERGY) {
            double v[1] = {e};
            block_sum<1>(v);
            if (tid == 0) epart[blockIdx.x] = v[0];
        }
        __syncthreads();
    }
    if (mode & MESH_INV) {
        if constexpr (KC > 0 && TWC > 0)
            fft_ct<KC, TWC, TWC, NT, true>(buf, tw, tid);
        else
            fft_lds(buf, ax1, twl, tw, true, tid, NT);
    }
    for (int t = tid; t < K1 * TW; t += NT) {
        const int c = t & (TW - 1), g1 = t >> twl;
        base[(size_t)g1 * K2 + c] = buf[t];
    }
}

// ------------------------------------------------------------------ pass 5
template <int KC, int TWC>
__global__ __launch_bounds__(NT) void k_c2r(KParams k, FftAxis ax3, const float2* __restrict__ C,
                                           float* __restrict__ R, const int* __restrict__ done) {
    if (done && *done) return;
    extern __shared__ float2 sm[];
    const int K3 = KC ? KC : k.K3;
    const int TW = TWC ? TWC : k.TW;
    const int K3h = K3 / 2 + 1;
    const int K1 = k.K1, K2 = k.K2;
    const int ncol = TW >> 1;
    const int twl = ilog2_dev(TW);
    const int ncl = twl - 1;
    float2* tw = sm;
    float2* X = sm + K3;
    float2* Z = X + K3h * TW;
    const int tid = threadIdx.x;
    const int g1 = blockIdx.x / k.ntile;
    const int g20 = (blockIdx.x - g1 * k.ntile) * TW;
    {
        auto ld_tw = [&](int t) { return ax3.tw[t]; };
        auto st_tw = [&](int t, float2 v) { tw[t] = v; };
        auto ld = [&](int t) {
            const int r = t & (TW - 1), m = t >> twl;
            return C[((size_t)m * K1 + g1) * K2 + g20 + r];
        };
        auto st = [&](int t, float2 v) { X[t] = v; };
        if constexpr (KC > 0 && TWC > 0) {
            stage2_ct<KC, (KC / 2 + 1) * TWC, NT, float2>(tid, ld_tw, st_tw, ld, st);
        } else {
            stage_rt<4, float2>(K3, tid, NT, ld_tw, st_tw);
            stage_rt<4, float2>(K3h * TW, tid, NT, ld, st);
        }
    }
    __syncthreads();
    // Z = X_even + i X_odd over the full axis (Hermitian extension)
    for (int t = tid; t < K3 * ncol; t += NT) {
        const int pr = t & (ncol - 1), m = t >> ncl;
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
    if constexpr (KC > 0 && TWC > 0)
        fft_ct<KC, TWC / 2, TWC / 2, NT, true>(Z, tw, tid);
    else
        fft_lds(Z, ax3, ncl, tw, true, tid, NT);
    const float* zf = reinterpret_cast<const float*>(Z);
    for (int t = tid; t < TW * K3; t += NT) {
        const int r = t / K3;
        const int g3 = t - r * K3;
        R[((size_t)g1 * K2 + g20 + r) * K3 + g3] = zf[(g3 * ncol + (r >> 1)) * 2 + (r & 1)];
    }
}

// ------------------------------------------------------------------ pass 5 fused with interpolation
// The complex-to-real pass of a (g1, TW-row) tile followed, while the tile's
// potential is still in LDS, by the part of every atom's back-interpolation
// (eq. matvec: the integral of the potential over the atom's charge
// distribution, here sum_g theta_i(g) phi(g)) that falls on this tile, so the
// real grid is never written or read again:
//   partial = w1(k1) sum_{k2: row in tile} w2(k2) sum_k3 w3(k3) phi(g1, h2 - k2, h3 - k3)
// for every atom with h1 = g1 + k1 (k1 < p) whose rows h2 - p + 1 .. h2 meet
// the tile (TW >= p - 1, so at most two tiles).  Each partial goes to its own
// slot, mpart[(2 k1 + t) n + atom] with t = 0 for the tile holding row h2 and
// t = 1 for the tile before it (written as 0 by the first when the atom's rows
// all lie in one tile): 2p FP32 partials per atom, summed in a fixed order by
// the pair-product kernel, so the result does not depend on block timing.
template <int KC, int TWC, int PC>
__global__ __launch_bounds__(NT) void k_c2r_interp(KParams k, FftAxis ax3, const float2* __restrict__ C,
                                                  const int* __restrict__ bin_start,
                                                  const int* __restrict__ home,
                                                  const float* __restrict__ wts, float* __restrict__ mpart,
                                                  const int* __restrict__ done) {
    if (done && *done) return;
    extern __shared__ float2 sm[];
    constexpr bool CT = KC > 0 && TWC > 0;
    const int K3 = KC ? KC : k.K3;
    const int TW = TWC ? TWC : k.TW;
    const int p = PC ? PC : k.p;
    const int K3h = K3 / 2 + 1;
    const int K1 = k.K1, K2 = k.K2;
    const int ncol = TW >> 1;
    const int twl = ilog2_dev(TW);
    const int ncl = twl - 1;
    float2* tw = sm;
    float2* X = sm + K3;
    // compile-time sizes: the packed rows Z (K3 x TW/2) replace X (K3/2 + 1
    // rows of TW) in place through registers, halving the block's LDS
    float2* Z = CT ? X : X + K3h * TW;
    __shared__ int seg_lo[2 * QEQ_MAXP], seg_len[2 * QEQ_MAXP], seg_off[2 * QEQ_MAXP + 1];
    const int tid = threadIdx.x;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int g1 = blk / k.ntile;
    const int g20 = (blk - g1 * k.ntile) * TW;
    // candidate segments (as in the spread pass): homes h1 = g1 + k1,
    // h2 in [g20, g20 + TW + p - 1), two pieces when the range wraps
    if (tid < p) {
        const int k1 = tid;
        int h1 = g1 + k1;
        if (h1 >= K1) h1 -= K1;
        const int b0 = h1 * K2;
        const int hi = g20 + TW + p - 1;
        const int e1 = hi < K2 ? hi : K2;
        const int lo0 = bin_start[b0 + g20];
        seg_lo[2 * k1] = lo0;
        seg_len[2 * k1] = bin_start[b0 + e1] - lo0;
        if (hi > K2) {
            const int lo1 = bin_start[b0];
            seg_lo[2 * k1 + 1] = lo1;
            seg_len[2 * k1 + 1] = bin_start[b0 + (hi - K2)] - lo1;
        } else {
            seg_lo[2 * k1 + 1] = 0;
            seg_len[2 * k1 + 1] = 0;
        }
    }
    {
        auto ld_tw = [&](int t) { return ax3.tw[t]; };
        auto st_tw = [&](int t, float2 v) { tw[t] = v; };
        auto ld = [&](int t) {
            const int r = t & (TW - 1), m = t >> twl;
            return C[((size_t)m * K1 + g1) * K2 + g20 + r];
        };
        auto st = [&](int t, float2 v) { X[t] = v; };
        if constexpr (CT) {
            stage2_ct<KC, (KC / 2 + 1) * TWC, NT, float2>(tid, ld_tw, st_tw, ld, st);
        } else {
            stage_rt<4, float2>(K3, tid, NT, ld_tw, st_tw);
            stage_rt<4, float2>(K3h * TW, tid, NT, ld, st);
        }
    }
    __syncthreads();
    if (tid == 0) {
        int off = 0;
        for (int sg = 0; sg < 2 * p; ++sg) {
            seg_off[sg] = off;
            off += seg_len[sg];
        }
        seg_off[2 * p] = off;
    }
    // Z = X_even + i X_odd over the full axis (Hermitian extension)
    auto zval = [&](int t) {
        const int pr = t & (ncol - 1), m = t >> ncl;
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
        return make_float2(xa.x - xb.y, xa.y + xb.x);
    };
    // compile-time sizes: the packed values are built inside the first radix
    // stage of the transform (each item reads the X elements of its R0 inputs
    // into registers; after the barrier the stage's outputs overwrite X in
    // place), so the packing costs no LDS pass of its own
    constexpr int NCZ = CT ? TWC / 2 : 1;
    constexpr int R0 = CT ? ct_radix_at(KC, 0, TWC / 2, NT) : 1;
    constexpr int PER0 = CT ? KC / R0 : 1;
    constexpr int IT0 = CT ? (PER0 * NCZ + NT - 1) / NT : 1;
    float2 v0[IT0][R0];
    if constexpr (CT) {
#pragma unroll
        for (int it = 0; it < IT0; ++it) {
            const int item = tid + it * NT;
            if ((PER0 * NCZ) % NT == 0 || item < PER0 * NCZ) {
                const int c = item % NCZ, j = item / NCZ;
#pragma unroll
                for (int r = 0; r < R0; ++r) v0[it][r] = zval((j + r * PER0) * NCZ + c);
            }
        }
    } else {
        for (int t = tid; t < K3 * ncol; t += NT) Z[t] = zval(t);
    }
    __syncthreads();
    // the first round's candidate is fetched before the transform so that its
    // loads overlap it
    const int ncand = seg_off[2 * p];
    const int n = k.n;
    constexpr int PM = PC ? PC : QEQ_MAXP;
    float w1 = 0.f, w2[PM], w3[PM];
    int a = 0, k1 = 0, h2 = 0, h3 = 0;
    auto load_cand = [&](int cidx) {
        // last segment starting at or before cidx (empty segments are passed over)
        int sg = 0;
#pragma unroll
        for (int s2 = 1; s2 < 2 * PM; ++s2) {
            if (!PC && s2 >= 2 * p) break;
            sg += cidx >= seg_off[s2] ? 1 : 0;
        }
        k1 = sg >> 1;
        a = seg_lo[sg] + (cidx - seg_off[sg]);
        const float* w = wts + (size_t)a * 3 * QEQ_MAXP;
        w1 = w[k1];
#pragma unroll
        for (int kk = 0; kk < PM; ++kk) {
            if (!PC && kk >= p) break;
            w2[kk] = w[QEQ_MAXP + kk];
            w3[kk] = w[2 * QEQ_MAXP + kk];
        }
        h2 = home[4 * a + 1];
        h3 = home[4 * a + 2];
    };
    if (tid < ncand) load_cand(tid);
    if constexpr (CT) {
#pragma unroll
        for (int it = 0; it < IT0; ++it) {
            const int item = tid + it * NT;
            if ((PER0 * NCZ) % NT == 0 || item < PER0 * NCZ) {
                const int c = item % NCZ, j = item / NCZ;
                dft<R0>(v0[it], true);
#pragma unroll
                for (int r = 0; r < R0; ++r) Z[(j * R0 + r) * NCZ + c] = v0[it][r];
            }
        }
        __syncthreads();
        fft_ct<KC, TWC / 2, TWC / 2, NT, true, 1, R0>(Z, tw, tid);
    } else {
        fft_lds(Z, ax3, ncl, tw, true, tid, NT);
    }
    // phi(g1, g20 + r, g3) = zf[(g3 ncol + r / 2) 2 + r % 2]
    const float* zf = reinterpret_cast<const float*>(Z);
    for (int cidx = tid; cidx < ncand; cidx += NT) {
        if (cidx != tid) load_cand(cidx);
        int d = h2 - g20;
        if (d < 0) d += K2;
        float s = 0.f;
#pragma unroll
        for (int k2 = 0; k2 < PM; ++k2) {
            if (!PC && k2 >= p) break;
            const int r = d - k2;
            if (r < 0 || r >= TW) continue;
            const float* zr = zf + (r >> 1) * 2 + (r & 1);
            float t = 0.f;
#pragma unroll
            for (int k3 = 0; k3 < PM; ++k3) {
                if (!PC && k3 >= p) break;
                int g3 = h3 - k3;
                if (g3 < 0) g3 += K3;
                t += w3[k3] * zr[g3 * ncol * 2];
            }
            s += w2[k2] * t;
        }
        const int slot = 2 * k1 + (d < TW ? 0 : 1);
        mpart[(size_t)slot * n + a] = w1 * s;
        if (d < TW && d >= p - 1) mpart[(size_t)(slot + 1) * n + a] = 0.f;
    }
}

// ------------------------------------------------------------------ passes 1 + 2 fused
// Spread, axis-3 real-to-complex and axis-2 forward transforms of one g1
// plane in LDS, for grids whose plane half spectrum K2 (K3/2 + 1) fits (one
// block per CU): the mirror image of k_slab_inv, saving the grid round trip
// between the spread and the axis-2 pass.
//   Candidates: the atoms whose home plane h1 = g1 + k1 (k1 < p) reaches g1,
//   one index range per k1 (atoms are sorted by home bin), taken by the
//   block's threads together and held in registers (CPT per thread).
//   Fixed point, one scale per row g2: every value of row g2 is a sum of one
//   term per candidate whose axis-2 support covers the row, so |value| <=
//   S(g2) = sum of |src| w1(k1) max(w2) max(w3) over those candidates.  The
//   plane total S (< 2^eS) fixes a quantum U = 2^(eS - 20); each candidate
//   adds floor(bound / U) + 1 to the integer bounds of its p rows (integer
//   sums: order-independent), so S(g2) <= rb(g2) U, and the row is scaled by
//   2^(30 - e) with rb(g2) U < 2^e.  A row's bound sums over about p / K2 of
//   the plane's candidates (about 32 of 1,024 at 192^3 and 32,768 atoms), a
//   row tile's of k_spread_r2c over about (TW + p - 1) / K2 of them, so the
//   row scales are finer.
//   Then two real rows per complex line for the axis-3 transform (the
//   conversion inside its first radix stage), their half spectra unpacked
//   to X[g2][m3] (row stride K3/2 + 1), the axis-2 transform of every m3
//   column, and C[m3][g1][m2] written.
constexpr int PLANE_NT = 1024;

template <int K2C, int K3C>
__global__ __launch_bounds__(PLANE_NT) void k_plane_fwd(KParams k, FftAxis ax2, FftAxis ax3,
                                                       const double* __restrict__ src,
                                                       const int* __restrict__ bin_start,
                                                       const int* __restrict__ home,
                                                       const float* __restrict__ wts, float2* __restrict__ C,
                                                       const int* __restrict__ done) {
    constexpr int P = 6, CPT = 2;
    constexpr int KS = K3C / 2 + 1;   // complex row stride of X
    constexpr int AS = K3C + 1;       // int row stride of the accumulator
    constexpr int NP = K2C / 2;       // row pairs
    static_assert(K2C * AS * 4 <= K2C * KS * 8, "accumulator must fit the plane buffer");
    static_assert(K3C * NP <= K2C * KS, "packed rows must fit the plane buffer");
    extern __shared__ float2 sm[];
    float2* tw2 = sm;              // K2C: e^{-2 pi i j / K2}
    float2* tw3 = tw2 + K2C;       // K3C: e^{-2 pi i j / K3}
    float2* X = tw3 + K3C;         // K2C x KS
    int* acc = reinterpret_cast<int*>(X);
    __shared__ int rb[K2C];
    __shared__ float rinv[K2C], rsc[K2C];
    __shared__ int sh_e;
    const int tid = threadIdx.x;
    // XCD-aware plane order: the p planes that read one atom run on one XCD
    const int g1 = xcd_remap(blockIdx.x, gridDim.x);
    const int K1 = k.K1;
    // twiddles and the candidate ranges are requested before the converged
    // flag is examined, so the loads share one round trip
    constexpr int NTW = K2C + K3C;
    float2 twv = make_float2(0.f, 0.f);
    if (tid < NTW) twv = tid < K2C ? ax2.tw[tid] : ax3.tw[tid - K2C];
    int blo[P], bhi[P];
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1) {
        int h1 = g1 + k1;
        if (h1 >= K1) h1 -= K1;
        blo[k1] = bin_start[h1 * K2C];
        bhi[k1] = bin_start[(h1 + 1) * K2C];
    }
    if (done && *done) return;
    if (tid < NTW) sm[tid] = twv;
    {
        int4* a4 = reinterpret_cast<int4*>(acc);
        constexpr int N4 = K2C * AS / 4;
        static_assert((K2C * AS) % 4 == 0, "accumulator clears as int4");
        for (int t = tid; t < N4; t += PLANE_NT) a4[t] = make_int4(0, 0, 0, 0);
    }
    if (tid < K2C) rb[tid] = 0;
    int off[P + 1];
    off[0] = 0;
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1) off[k1 + 1] = off[k1] + (bhi[k1] - blo[k1]);
    const int ncand = off[P];
    // candidate t: plane k1 (the last range starting at or before t), atom a
    float a0[CPT], w2[CPT][P], w3[CPT][P];
    double bnd[CPT];
    int h2[CPT], h3[CPT];
    auto load = [&](int s, int t) {
        int k1 = 0, a = blo[0] + t;
#pragma unroll
        for (int u = 1; u < P; ++u) {
            if (t >= off[u]) {
                k1 = u;
                a = blo[u] + (t - off[u]);
            }
        }
        const float* w = wts + (size_t)a * 3 * QEQ_MAXP;
        const double sv = src[a];
        const float w1 = w[k1];
        a0[s] = (float)sv * w1;
        float m2 = 0.f, m3 = 0.f;
#pragma unroll
        for (int kk = 0; kk < P; ++kk) {
            w2[s][kk] = w[QEQ_MAXP + kk];
            w3[s][kk] = w[2 * QEQ_MAXP + kk];
            m2 = fmaxf(m2, w2[s][kk]);
            m3 = fmaxf(m3, w3[s][kk]);
        }
        bnd[s] = fabs((double)a0[s]) * (double)m2 * (double)m3;
        h2[s] = home[4 * a + 1];
        h3[s] = home[4 * a + 2];
    };
    const int nround = (ncand + CPT * PLANE_NT - 1) / (CPT * PLANE_NT);
    // pass A: the plane bound S (candidates of later rounds are loaded again
    // in the passes below; one round keeps them in registers)
    {
        double v[1] = {0.0};
        for (int rd = 0; rd < nround; ++rd) {
#pragma unroll
            for (int s = 0; s < CPT; ++s) {
                const int t = (rd * CPT + s) * PLANE_NT + tid;
                if (t < ncand) {
                    load(s, t);
                    v[0] += bnd[s];
                }
            }
        }
        block_sum<1>(v);   // its barriers also order the clears above
        if (tid == 0) {
            int e = 0;
            (void)frexp(v[0] > 0.0 ? v[0] : 1.0, &e);   // S < 2^e
            sh_e = e;
        }
        __syncthreads();
    }
    const int eS = sh_e;
    // pass B: integer row bounds in units of U = 2^(eS - 20); each term is
    // below 2^20 and the terms of a row sum to below 2^20 + ncand
    for (int rd = 0; rd < nround; ++rd) {
#pragma unroll
        for (int s = 0; s < CPT; ++s) {
            const int t = (rd * CPT + s) * PLANE_NT + tid;
            if (t < ncand) {
                if (nround > 1) load(s, t);
                const int q = (int)ldexp(bnd[s], 20 - eS) + 1;
#pragma unroll
                for (int k2 = 0; k2 < P; ++k2) {
                    int r = h2[s] - k2;
                    if (r < 0) r += K2C;
                    atomicAdd(rb + r, q);
                }
            }
        }
    }
    __syncthreads();
    if (tid < K2C) {
        int e = 0;
        const double sr = ldexp((double)rb[tid], eS - 20);
        (void)frexp(sr > 0.0 ? sr : 1.0, &e);   // S(g2) <= sr < 2^e
        const int x = max(-126, min(126, 30 - e));
        rsc[tid] = ldexpf(1.0f, x);
        rinv[tid] = ldexpf(1.0f, -x);
    }
    __syncthreads();
    // pass C: terms rounded to integers by one FP64 fused multiply-add with
    // 1.5 * 2^52 (the low word of the sum is the two's-complement integer)
    constexpr double RND = 6755399441055744.0;
    for (int rd = 0; rd < nround; ++rd) {
#pragma unroll
        for (int s = 0; s < CPT; ++s) {
            const int t = (rd * CPT + s) * PLANE_NT + tid;
            if (t < ncand) {
                if (nround > 1) load(s, t);
                double w3d[P];
                int col[P];
#pragma unroll
                for (int k3 = 0; k3 < P; ++k3) {
                    w3d[k3] = (double)w3[s][k3];
                    int g3 = h3[s] - k3;
                    if (g3 < 0) g3 += K3C;
                    col[k3] = g3;
                }
#pragma unroll
                for (int k2 = 0; k2 < P; ++k2) {
                    int r = h2[s] - k2;
                    if (r < 0) r += K2C;
                    const double a1 = (double)(a0[s] * rsc[r]) * (double)w2[s][k2];   // exact
                    int* row = acc + r * AS;
#pragma unroll
                    for (int k3 = 0; k3 < P; ++k3) {
                        const int v = (int)(unsigned)__double_as_longlong(fma(a1, w3d[k3], RND));
                        atomicAdd(row + col[k3], v);
                    }
                }
            }
        }
    }
    __syncthreads();
    // rows 2c and 2c + 1 as one complex line along g3 (Z[g3][c], c < NP):
    // the conversion to FP32 inside the first radix stage
    float2* Z = X;
    {
        constexpr int R0 = ct_radix_at(K3C, 0, NP, PLANE_NT), PER0 = K3C / R0;
        constexpr int ITEMS = PER0 * NP, IT0 = (ITEMS + PLANE_NT - 1) / PLANE_NT;
        float2 v[IT0][R0];
#pragma unroll
        for (int it = 0; it < IT0; ++it) {
            const int item = tid + it * PLANE_NT;
            if (ITEMS % PLANE_NT == 0 || item < ITEMS) {
                const int c = item % NP, j = item / NP;
                const int* re = acc + (2 * c) * AS;
                const int* im = re + AS;
                const float se = rinv[2 * c], so = rinv[2 * c + 1];
#pragma unroll
                for (int r = 0; r < R0; ++r) {
                    const int g3 = j + r * PER0;
                    v[it][r] = make_float2((float)re[g3] * se, (float)im[g3] * so);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < IT0; ++it) {
            const int item = tid + it * PLANE_NT;
            if (ITEMS % PLANE_NT == 0 || item < ITEMS) {
                const int c = item % NP, j = item / NP;
                dft<R0>(v[it], false);
#pragma unroll
                for (int r = 0; r < R0; ++r) Z[(j * R0 + r) * NP + c] = v[it][r];
            }
        }
        __syncthreads();
        fft_ct<K3C, NP, NP, PLANE_NT, false, 1, R0>(Z, tw3, tid);
    }
    // unpack the two rows' half spectra, m3 = 0 .. K3/2: every LDS read of the
    // thread first (the rows overwrite the packed lines)
    {
        constexpr int NI = NP * KS, PI = (NI + PLANE_NT - 1) / PLANE_NT;
        float2 za[PI], zb[PI];
#pragma unroll
        for (int u = 0; u < PI; ++u) {
            const int t = tid + u * PLANE_NT;
            if (NI % PLANE_NT == 0 || t < NI) {
                const int m = t / NP, c = t - m * NP;
                za[u] = Z[m * NP + c];
                zb[u] = Z[(m == 0 ? 0 : K3C - m) * NP + c];
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PI; ++u) {
            const int t = tid + u * PLANE_NT;
            if (NI % PLANE_NT == 0 || t < NI) {
                const int m = t / NP, c = t - m * NP;
                const float2 Zv = za[u], Zc = make_float2(zb[u].x, -zb[u].y);
                const float2 d = csub(Zv, Zc);
                X[(2 * c) * KS + m] = make_float2(0.5f * (Zv.x + Zc.x), 0.5f * (Zv.y + Zc.y));
                X[(2 * c + 1) * KS + m] = make_float2(0.5f * d.y, -0.5f * d.x);
            }
        }
        __syncthreads();
    }
    // axis-2 transform of every m3 column, then C[m3][g1][m2]
    fft_ct<K2C, KS, KS, PLANE_NT, false>(X, tw2, tid);
    __syncthreads();
#pragma unroll 4
    for (int t = tid; t < KS * K2C; t += PLANE_NT) {
        const int m3 = t / K2C, m2 = t - m3 * K2C;
        C[((size_t)m3 * K1 + g1) * K2C + m2] = X[m2 * KS + m3];
    }
}

// ------------------------------------------------------------------ passes 4 + 5 fused
// Inverse axis-2 and axis-3 complex-to-real transforms of one g1 slab in LDS,
// for grids whose slab half spectrum K2 (K3/2 + 1) fits (one block per CU):
//   load C[m3][g1][m2] as X[m2][m3] (row stride KS = K3/2 + 1),
//   inverse FFT along m2 for all K3/2 + 1 columns -> X[g2][m3],
//   each row g2: the real inverse DFT of length N = K3 from its half spectrum
//   as one complex inverse FFT of length N/2, in place:
//     E[k] = X[k] + conj X[N/2 - k],  O[k] = e^{2 pi i k/N} (X[k] - conj X[N/2 - k]),
//     z = IFFT_{N/2}(E + i O),  x[2n] = Re z[n],  x[2n + 1] = Im z[n]
//   (both IFFT(E) and IFFT(O) are real because the line is),
//   store R[g1][g2][g3] as pairs.  Saves the grid round trip between the two
//   separate passes.
//   INTERP: instead of storing the slab, every atom whose spline support meets
//   plane g1 (h1 = g1 + k1, k1 < p) takes its partial back-interpolation
//   w1(k1) sum_k2 w2(k2) sum_k3 w3(k3) phi(g1, h2 - k2, h3 - k3) from the slab
//   in LDS into slot 2 k1 of mpart (slot 2 k1 + 1 = 0: the whole plane is
//   here), as the fused tile pass does.
constexpr int SLAB_NT = 1024;

template <int K2C, int K3C, bool INTERP = false>
__global__ __launch_bounds__(SLAB_NT) void k_slab_inv(KParams k, FftAxis ax2, FftAxis ax3,
                                                     const float2* __restrict__ C, float* __restrict__ R,
                                                     const int* __restrict__ done,
                                                     const int* __restrict__ bin_start = nullptr,
                                                     const int* __restrict__ home = nullptr,
                                                     const float* __restrict__ wts = nullptr,
                                                     float* __restrict__ mpart = nullptr) {
    if (done && *done) return;
    constexpr int K3H = K3C / 2 + 1;
    constexpr int KS = K3H;
    constexpr int NH = K3C / 2;
    extern __shared__ float2 sm[];
    float2* tw2 = sm;            // K2C: e^{-2 pi i j / K2}
    float2* tw3 = tw2 + K2C;     // K3C: e^{-2 pi i j / K3}
    float2* twh = tw3 + K3C;     // NH:  e^{-2 pi i j / NH}
    float2* X = twh + NH;        // K2C x KS
    const int tid = threadIdx.x;
    // XCD-aware plane order: the p planes that read one atom's weights run
    // on the same XCD and share its L2
    const int g1 = xcd_remap(blockIdx.x, gridDim.x);
    const int K1 = k.K1;
    // interpolation: atom ranges of the p planes whose support reaches g1
    // (read now, used at the end)
    constexpr int P = 6;
    int blo[P], bhi[P];
    if constexpr (INTERP) {
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1) {
            int h1 = g1 + k1;
            if (h1 >= K1) h1 -= K1;
            blo[k1] = bin_start[h1 * K2C];
            bhi[k1] = bin_start[(h1 + 1) * K2C];
        }
    }
    // The three twiddle tables (K2C + K3C + NH entries) and the plane, in two
    // groups of m3 columns: the axis-2 transforms of the first group run
    // while the second group's loads are in flight (barriers wait on LDS
    // only), and the columns are independent.
    constexpr int CA = (K3H + 1) / 2, CB = K3H - CA;
    auto ld_col = [&](int m3, int m2) { return C[((size_t)m3 * K1 + g1) * K2C + m2]; };
    {
        auto ld_tw = [&](int t) {
            return t < K2C ? ax2.tw[t] : (t < K2C + K3C ? ax3.tw[t - K2C] : ax3.tw[2 * (t - K2C - K3C)]);
        };
        auto st_tw = [&](int t, float2 v) { tw2[t] = v; };   // tw2 | tw3 | twh are contiguous
        auto ld = [&](int t) {
            const int m3 = t / K2C, m2 = t - m3 * K2C;
            return ld_col(m3, m2);
        };
        auto st = [&](int t, float2 v) {
            const int m3 = t / K2C, m2 = t - m3 * K2C;
            X[m2 * KS + m3] = v;
        };
        stage2_ct<K2C + K3C + NH, CA * K2C, SLAB_NT, float2>(tid, ld_tw, st_tw, ld, st);
    }
    constexpr int PB = (CB * K2C + SLAB_NT - 1) / SLAB_NT;
    float2 vb[PB];
#pragma unroll
    for (int u = 0; u < PB; ++u) {
        const int t = tid + u * SLAB_NT;
        if ((CB * K2C) % SLAB_NT == 0 || t < CB * K2C) {
            const int m3 = t / K2C, m2 = t - m3 * K2C;
            vb[u] = ld_col(CA + m3, m2);
        }
    }
    __syncthreads();
    fft_ct<K2C, CA, KS, SLAB_NT, true>(X, tw2, tid);
#pragma unroll
    for (int u = 0; u < PB; ++u) {
        const int t = tid + u * SLAB_NT;
        if ((CB * K2C) % SLAB_NT == 0 || t < CB * K2C) {
            const int m3 = t / K2C, m2 = t - m3 * K2C;
            X[m2 * KS + CA + m3] = vb[u];
        }
    }
    __syncthreads();
    fft_ct<K2C, CB, KS, SLAB_NT, true>(X + CA, tw2, tid);
    // Length-NH inverse transform along each row g2 of the packed sequence
    // z(n) = (X(n) + conj X(NH - n)) + i (X(n) - conj X(NH - n)) e^{2 pi i n / K3}
    // (two real outputs per complex one).  Its first radix stage builds z
    // while loading: each item reads its R0 elements and their mirrors, so the
    // pairing costs no pass of its own over the plane.
    {
        constexpr int R0 = ct_radix_at(NH, 0, K2C, SLAB_NT);
        constexpr int PER0 = NH / R0;
        constexpr int ITEMS = PER0 * K2C;
        constexpr int IT0 = (ITEMS + SLAB_NT - 1) / SLAB_NT;
        float2 v[IT0][R0];
#pragma unroll
        for (int it = 0; it < IT0; ++it) {
            const int item = tid + it * SLAB_NT;
            if (ITEMS % SLAB_NT == 0 || item < ITEMS) {
                const int c = item % K2C, j = item / K2C;
                const float2* row = X + c * KS;
#pragma unroll
                for (int r = 0; r < R0; ++r) {
                    const int idx = j + r * PER0;
                    const float2 xk = row[idx], xq = row[NH - idx];
                    const float2 cq = make_float2(xq.x, -xq.y);
                    const float2 e = cadd(xk, cq);
                    float2 w = tw3[idx];
                    w.y = -w.y;
                    const float2 o = cmul(csub(xk, cq), w);
                    v[it][r] = make_float2(e.x - o.y, e.y + o.x);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < IT0; ++it) {
            const int item = tid + it * SLAB_NT;
            if (ITEMS % SLAB_NT == 0 || item < ITEMS) {
                const int c = item % K2C, j = item / K2C;
                dft<R0>(v[it], true);
                float2* row = X + c * KS;
#pragma unroll
                for (int r = 0; r < R0; ++r) row[j * R0 + r] = v[it][r];
            }
        }
        __syncthreads();
        fft_ct<NH, K2C, 1, SLAB_NT, true, 1, R0, KS>(X, twh, tid);
    }
    if constexpr (!INTERP) {
        float2* R2 = reinterpret_cast<float2*>(R) + (size_t)g1 * K2C * NH;
        for (int t = tid; t < K2C * NH; t += SLAB_NT) {
            const int g2 = t / NH, n = t - g2 * NH;
            R2[t] = X[g2 * KS + n];
        }
    } else {
        // phi(g1, g2, g3) = xf[2 KS g2 + g3].  The atoms of the p planes form
        // one index range (plane k1's atoms from off[k1]), so the block's
        // threads take them all at once: one round of atom loads, not p.
        const float* xf = reinterpret_cast<const float*>(X);
        const int n = k.n;
        int off[P + 1];
        off[0] = 0;
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1) off[k1 + 1] = off[k1] + (bhi[k1] - blo[k1]);
        for (int t = tid; t < off[P]; t += SLAB_NT) {
            int k1 = 0, a = blo[0] + t;
#pragma unroll
            for (int u = 1; u < P; ++u) {
                if (t >= off[u]) {
                    k1 = u;
                    a = blo[u] + (t - off[u]);
                }
            }
            {
                const float* w = wts + (size_t)a * 3 * QEQ_MAXP;
                const int h2 = home[4 * a + 1];
                const int h3 = home[4 * a + 2];
                float s = 0.f;
#pragma unroll
                for (int k2 = 0; k2 < P; ++k2) {
                    int g2 = h2 - k2;
                    if (g2 < 0) g2 += K2C;
                    const float* row = xf + 2 * KS * g2;
                    float r3 = 0.f;
#pragma unroll
                    for (int k3 = 0; k3 < P; ++k3) {
                        int g3 = h3 - k3;
                        if (g3 < 0) g3 += K3C;
                        r3 += w[2 * QEQ_MAXP + k3] * row[g3];
                    }
                    s += w[QEQ_MAXP + k2] * r3;
                }
                mpart[(size_t)(2 * k1) * n + a] = w[k1] * s;
                mpart[(size_t)(2 * k1 + 1) * n + a] = 0.f;
            }
        }
    }
}

__global__ void k_write_green(KParams k, float2* __restrict__ C, const float* __restrict__ b1,
                              const float* __restrict__ b2, const float* __restrict__ b3) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)k.K3h * k.K1 * k.K2;
    if (t >= total) return;
    const int m2 = (int)(t % k.K2);
    const int m1 = (int)((t / k.K2) % k.K1);
    const int m3 = (int)(t / ((size_t)k.K2 * k.K1));
    C[t] = make_float2(green_value(k, m1, m2, m3, b1, b2, b3), 0.f);
}

// Strain factor of one mode: under r -> (1 + eps) r (fractional coordinates
// fixed) k -> (1 + eps)^-T k and V -> (1 + tr eps) V, so
//   d ln G(m) / d eps_ab = -delta_ab + 2 (1/k^2 + eta^2/2) k_a k_b
// (the B-spline moduli do not change).  kv = 2 pi H^-1 m, returns k^2.
__device__ __forceinline__ float mode_kvec(const KParams& k, int m1, int m2, int m3, float kv[3]) {
    const float x1 = (float)(m1 <= k.K1 / 2 ? m1 : m1 - k.K1);
    const float x2 = (float)(m2 <= k.K2 / 2 ? m2 : m2 - k.K2);
    const float x3 = (float)m3;
    float k2 = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        kv[c] = 6.283185307179586477f * ((float)k.Hinv[c * 3] * x1 + (float)k.Hinv[c * 3 + 1] * x2 +
                                         (float)k.Hinv[c * 3 + 2] * x3);
        k2 += kv[c] * kv[c];
    }
    return k2;
}

// Component order of symmetric 3x3 tensors: 00, 11, 22, 01, 02, 12.
__device__ __forceinline__ void sym_pair(int comp, int& a, int& b) {
    a = comp < 3 ? comp : (comp == 5 ? 1 : 0);
    b = comp < 3 ? comp : (comp == 3 ? 1 : 2);
}

// G(m) d ln G / d eps_ab on the half spectrum: its inverse transform is the
// strain derivative of the mesh kernel Theta (for the self-correction term).
__global__ void k_write_green_strain(KParams k, float2* __restrict__ C, const float* __restrict__ b1,
                                     const float* __restrict__ b2, const float* __restrict__ b3, int comp) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)k.K3h * k.K1 * k.K2;
    if (t >= total) return;
    const int m2 = (int)(t % k.K2);
    const int m1 = (int)((t / k.K2) % k.K1);
    const int m3 = (int)(t / ((size_t)k.K2 * k.K1));
    const float g = green_value(k, m1, m2, m3, b1, b2, b3);
    float v = 0.f;
    if (g != 0.f) {
        float kv[3];
        const float k2 = mode_kvec(k, m1, m2, m3, kv);
        const float eta = (float)k.eta;
        int a, b;
        sym_pair(comp, a, b);
        v = g * ((a == b ? -1.f : 0.f) + 2.f * (1.f / k2 + 0.5f * eta * eta) * kv[a] * kv[b]);
    }
    C[t] = make_float2(v, 0.f);
}

// Virial of the reciprocal mesh energy E = 1/2 sum_m G(m) |Q(m)|^2: the
// axis-1 forward transform of a column tile (the grid already transformed
// along axes 3 and 2), then per mode e = G |Q|^2 (doubled off the m3 = 0
// plane) and per block the sums of e and of e c k_a k_b, c = 2 (1/k^2 + eta^2/2);
// W = 1/2 (sum e) delta - 1/2 sum e c k k.  The grid is left as it is.
template <int KC, int TWC>
__global__ __launch_bounds__(NT) void k_cols_virial(KParams k, FftAxis ax1, const float2* __restrict__ C,
                                                   const float* __restrict__ b1, const float* __restrict__ b2,
                                                   const float* __restrict__ b3, double* __restrict__ part) {
    extern __shared__ float2 sm[];
    const int K1 = KC ? KC : k.K1;
    const int TW = TWC ? TWC : k.TW;
    const int twl = ilog2_dev(TW);
    float2* tw = sm;
    float2* buf = sm + K1;
    const int tid = threadIdx.x;
    const int K2 = k.K2;
    const int m3 = blockIdx.x / k.ntile;
    const int g20 = (blockIdx.x - m3 * k.ntile) * TW;
    for (int t = tid; t < K1; t += NT) tw[t] = ax1.tw[t];
    const float2* base = C + (size_t)m3 * K1 * K2 + g20;
    for (int t = tid; t < K1 * TW; t += NT) {
        const int c = t & (TW - 1), g1 = t >> twl;
        buf[t] = base[(size_t)g1 * K2 + c];
    }
    __syncthreads();
    if constexpr (KC > 0 && TWC > 0)
        fft_ct<KC, TWC, TWC, NT, false>(buf, tw, tid);
    else
        fft_lds(buf, ax1, twl, tw, false, tid, NT);
    double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const float mult = (m3 == 0) ? 1.f : 2.f;
    const float eta = (float)k.eta;
    for (int t = tid; t < K1 * TW; t += NT) {
        const int c = t & (TW - 1), m1 = t >> twl;
        const float g = green_value(k, m1, g20 + c, m3, b1, b2, b3);
        if (g == 0.f) continue;
        const float2 x = buf[t];
        float kv[3];
        const float k2 = mode_kvec(k, m1, g20 + c, m3, kv);
        const float e = g * mult * (x.x * x.x + x.y * x.y);
        const float ec = e * 2.f * (1.f / k2 + 0.5f * eta * eta);
        v[0] += (double)e;
        v[1] += (double)(ec * kv[0] * kv[0]);
        v[2] += (double)(ec * kv[1] * kv[1]);
        v[3] += (double)(ec * kv[2] * kv[2]);
        v[4] += (double)(ec * kv[0] * kv[1]);
        v[5] += (double)(ec * kv[0] * kv[2]);
        v[6] += (double)(ec * kv[1] * kv[2]);
    }
    block_sum<7>(v);
    if (tid == 0)
        for (int u = 0; u < 7; ++u) part[(size_t)blockIdx.x * QEQ_NPART + u] = v[u];
}

size_t smem_spread(const KParams& k) {
    return sizeof(float2) * (size_t)k.K3 + sizeof(int) * (size_t)k.K3 * k.TWS;
}
size_t smem_rows(const KParams& k) { return sizeof(float2) * ((size_t)k.K2 + (size_t)k.K2 * (k.NR + 1)); }
size_t smem_cols(const KParams& k) { return sizeof(float2) * ((size_t)k.K1 + (size_t)k.K1 * k.TW); }
size_t smem_c2r(const KParams& k) {
    return sizeof(float2) * ((size_t)k.K3 + (size_t)k.K3h * k.TW + (size_t)k.K3 * (k.TW / 2));
}

// Specialised (length, tile) pairs; anything else runs the runtime-sized kernels.
#define QEQ_FOR_EACH_SIZE(X) X(24, 8) X(48, 16) X(96, 16) X(192, 16) X(320, 16) X(320, 8)
#define QEQ_FOR_EACH_SPREAD(X) \
    X(24, 8) X(48, 16) X(96, 16) X(192, 12) X(192, 16) X(192, 24) X(320, 8) X(320, 16)

int spread_pass(qeq_plan* pl, const double* src, const int* done) {
    const KParams& k = pl->kp;
    dim3 g(k.K1 * k.ntile_s), b(NT);
    const size_t sh = smem_spread(k);
    ProfScope ps(pl, PK_SPREAD_R2C);
    // the accumulator of long axes can exceed the default 64 KB window
#define X(KK, TT)                                                                                  \
    if (k.K3 == KK && k.TWS == TT && k.p == 6) {                                                    \
        if (sh > 65536)                                                                            \
            QEQ_HIP(hipFuncSetAttribute((const void*)k_spread_r2c<KK, TT, 6>,                      \
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));     \
        hipExtLaunchKernelGGL((k_spread_r2c<KK, TT, 6>), g, b, sh, pl->stream, ps.start(), ps.stop(), 0, k, \
                              pl->axes.ax[2], src, pl->bin_start, pl->home, pl->wts, pl->grid_c, done);   \
        return qeq_check(hipGetLastError());                                                       \
    }
    QEQ_FOR_EACH_SPREAD(X)
#undef X
    // the runtime-sized kernel indexes the tile by shifts: power-of-two widths only
    if (k.TWS & (k.TWS - 1)) return QEQ_EPLAN;
    if (sh > 65536)
        QEQ_HIP(hipFuncSetAttribute((const void*)k_spread_r2c<0, 0, 0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)sh));
    hipExtLaunchKernelGGL((k_spread_r2c<0, 0, 0>), g, b, sh, pl->stream, ps.start(), ps.stop(), 0, k,
                          pl->axes.ax[2], src, pl->bin_start, pl->home, pl->wts, pl->grid_c, done);
    return qeq_check(hipGetLastError());
}

template <bool INV>
int rows_pass_t(qeq_plan* pl, const int* done) {
    const KParams& k = pl->kp;
    const int nrows = k.K3h * k.K1;
    dim3 g((nrows + k.NR - 1) / k.NR), b(NT);
    const size_t sh = smem_rows(k);
    ProfScope ps(pl, INV ? PK_ROWS_INV : PK_ROWS_FWD);
#define X(KK, TT)                                                                                  \
    if (k.K2 == KK && k.NR == 16) {                                                                \
        hipExtLaunchKernelGGL((k_fft_rows<KK, 16, INV>), g, b, sh, pl->stream, ps.start(), ps.stop(), 0, \
                              k, pl->axes.ax[1], pl->grid_c, nrows, done);                          \
        return qeq_check(hipGetLastError());                                                       \
    }
    QEQ_FOR_EACH_SIZE(X)
#undef X
#define X(KK)                                                                                      \
    if (k.K2 == KK && k.NR == 4) {                                                                 \
        hipExtLaunchKernelGGL((k_fft_rows<KK, 4, INV>), g, b, sh, pl->stream, ps.start(), ps.stop(), 0, \
                              k, pl->axes.ax[1], pl->grid_c, nrows, done);                          \
        return qeq_check(hipGetLastError());                                                       \
    }
    X(320)
#undef X
    hipExtLaunchKernelGGL((k_fft_rows<0, 0, INV>), g, b, sh, pl->stream, ps.start(), ps.stop(), 0, k,
                          pl->axes.ax[1], pl->grid_c, nrows, done);
    return qeq_check(hipGetLastError());
}

int rows_pass(qeq_plan* pl, int inv, const int* done) {
    return inv ? rows_pass_t<true>(pl, done) : rows_pass_t<false>(pl, done);
}

int cols_pass(qeq_plan* pl, int mode, double* epart, const int* done) {
    const KParams& k = pl->kp;
    dim3 g(k.K3h * k.ntile), b(NT);
    const size_t sh = smem_cols(k);
    ProfScope ps(pl, PK_COLS_GREEN);
    // Gaussian-on-grid densities carry no B-spline moduli
    const float* b1 = pl->pw_active ? pl->pw_ones : pl->bmod[0];
    const float* b2 = pl->pw_active ? pl->pw_ones : pl->bmod[1];
    const float* b3 = pl->pw_active ? pl->pw_ones : pl->bmod[2];
#define X(KK, TT)                                                                                  \
    if (k.K1 == KK && k.TW == TT) {                                                                \
        hipExtLaunchKernelGGL((k_fft_cols<KK, TT>), g, b, sh, pl->stream, ps.start(), ps.stop(), 0, k,   \
                              pl->axes.ax[0], pl->grid_c, b1, b2, b3, mode, epart, done);           \
        return qeq_check(hipGetLastError());                                                       \
    }
    QEQ_FOR_EACH_SIZE(X)
#undef X
    hipExtLaunchKernelGGL((k_fft_cols<0, 0>), g, b, sh, pl->stream, ps.start(), ps.stop(), 0, k, pl->axes.ax[0],
                          pl->grid_c, b1, b2, b3, mode, epart, done);
    return qeq_check(hipGetLastError());
}

int cols_virial_pass(qeq_plan* pl, double* part) {
    const KParams& k = pl->kp;
    dim3 g(k.K3h * k.ntile), b(NT);
    const size_t sh = smem_cols(k);
#define X(KK, TT)                                                                                  \
    if (k.K1 == KK && k.TW == TT) {                                                                \
        hipLaunchKernelGGL((k_cols_virial<KK, TT>), g, b, sh, pl->stream, k, pl->axes.ax[0], pl->grid_c, \
                           pl->bmod[0], pl->bmod[1], pl->bmod[2], part);                            \
        return qeq_check(hipGetLastError());                                                       \
    }
    QEQ_FOR_EACH_SIZE(X)
#undef X
    hipLaunchKernelGGL((k_cols_virial<0, 0>), g, b, sh, pl->stream, k, pl->axes.ax[0], pl->grid_c, pl->bmod[0],
                       pl->bmod[1], pl->bmod[2], part);
    return qeq_check(hipGetLastError());
}

int c2r_pass(qeq_plan* pl, const int* done) {
    const KParams& k = pl->kp;
    dim3 g(k.K1 * k.ntile), b(NT);
    const size_t sh = smem_c2r(k);
    ProfScope ps(pl, PK_C2R);
#define X(KK, TT)                                                                                  \
    if (k.K3 == KK && k.TW == TT) {                                                                \
        hipExtLaunchKernelGGL((k_c2r<KK, TT>), g, b, sh, pl->stream, ps.start(), ps.stop(), 0, k,         \
                              pl->axes.ax[2], pl->grid_c, pl->grid_r, done);                        \
        return qeq_check(hipGetLastError());                                                       \
    }
    QEQ_FOR_EACH_SIZE(X)
#undef X
    hipExtLaunchKernelGGL((k_c2r<0, 0>), g, b, sh, pl->stream, ps.start(), ps.stop(), 0, k, pl->axes.ax[2],
                          pl->grid_c, pl->grid_r, done);
    return qeq_check(hipGetLastError());
}

// The complex-to-real pass fused with the back-interpolation (2p partials per
// atom in pl->mpart); needs TW >= p - 1 (at most two tiles per atom).
bool c2r_interp_available(const qeq_plan* pl) {
    const KParams& k = pl->kp;
    return pl->fused_interp && k.TW >= k.p - 1 && k.K2 >= k.TW + k.p - 1 && pl->mpart != nullptr;
}

int c2r_interp_pass(qeq_plan* pl, const int* done) {
    const KParams& k = pl->kp;
    dim3 g(k.K1 * k.ntile), b(NT);
    const size_t sh = smem_c2r(k);
    const size_t sh_ct = sizeof(float2) * ((size_t)k.K3 + (size_t)k.K3h * k.TW);   // Z in place of X
    ProfScope ps(pl, PK_C2R);
#define X(KK, TT)                                                                                  \
    if (k.K3 == KK && k.TW == TT && k.p == 6) {                                                     \
        hipExtLaunchKernelGGL((k_c2r_interp<KK, TT, 6>), g, b, sh_ct, pl->stream, ps.start(), ps.stop(), 0, k, \
                              pl->axes.ax[2], pl->grid_c, pl->bin_start, pl->home, pl->wts, pl->mpart, done); \
        return qeq_check(hipGetLastError());                                                       \
    }
    QEQ_FOR_EACH_SIZE(X)
#undef X
    hipExtLaunchKernelGGL((k_c2r_interp<0, 0, 0>), g, b, sh, pl->stream, ps.start(), ps.stop(), 0, k, pl->axes.ax[2],
                          pl->grid_c, pl->bin_start, pl->home, pl->wts, pl->mpart, done);
    return qeq_check(hipGetLastError());
}

size_t smem_slab(int K2, int K3) {
    return sizeof(float2) * ((size_t)K2 + K3 + K3 / 2 + (size_t)K2 * (K3 / 2 + 1));
}

// Lengths with a fused slab kernel; the slab must fit the LDS of one CU.
#define QEQ_FOR_EACH_SLAB(X) X(96, 96) X(192, 192)

bool slab_available(const qeq_plan* pl) {
    const KParams& k = pl->kp;
    if (!pl->fused_inverse || k.K1 < 64) return false;
#define X(A, B) if (k.K2 == A && k.K3 == B) return true;
    QEQ_FOR_EACH_SLAB(X)
#undef X
    return false;
}

int slab_interp_pass(qeq_plan* pl, const int* done) {
    const KParams& k = pl->kp;
    ProfScope ps(pl, PK_C2R);
#define X(A, B)                                                                                    \
    if (k.K2 == A && k.K3 == B && k.p == 6) {                                                      \
        const size_t sh = smem_slab(A, B);                                                         \
        QEQ_HIP(hipFuncSetAttribute((const void*)k_slab_inv<A, B, true>,                           \
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));         \
        hipExtLaunchKernelGGL((k_slab_inv<A, B, true>), dim3(k.K1), dim3(SLAB_NT), sh, pl->stream, ps.start(), \
                              ps.stop(), 0, k, pl->axes.ax[1], pl->axes.ax[2], pl->grid_c, pl->grid_r, done, \
                              pl->bin_start, pl->home, pl->wts, pl->mpart);                         \
        return qeq_check(hipGetLastError());                                                       \
    }
    QEQ_FOR_EACH_SLAB(X)
#undef X
    return QEQ_EPLAN;
}

bool slab_interp_available(const qeq_plan* pl) {
    return slab_available(pl) && pl->fused_interp && pl->kp.p == 6 && pl->mpart != nullptr;
}

int slab_inv_pass(qeq_plan* pl, const int* done) {
    const KParams& k = pl->kp;
    ProfScope ps(pl, PK_C2R);
#define X(A, B)                                                                                    \
    if (k.K2 == A && k.K3 == B) {                                                                  \
        const size_t sh = smem_slab(A, B);                                                         \
        QEQ_HIP(hipFuncSetAttribute((const void*)k_slab_inv<A, B>,                                 \
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));         \
        hipExtLaunchKernelGGL((k_slab_inv<A, B>), dim3(k.K1), dim3(SLAB_NT), sh, pl->stream, ps.start(), \
                              ps.stop(), 0, k, pl->axes.ax[1], pl->axes.ax[2], pl->grid_c, pl->grid_r, done, \
                              nullptr, nullptr, nullptr, nullptr);                                  \
        return qeq_check(hipGetLastError());                                                       \
    }
    QEQ_FOR_EACH_SLAB(X)
#undef X
    return QEQ_EPLAN;
}

// Lengths with a fused forward plane kernel (spread + axis-3 + axis-2).
#define QEQ_FOR_EACH_PLANE_FWD(X) X(192, 192)

size_t smem_plane_fwd(int K2, int K3) {
    return sizeof(float2) * ((size_t)K2 + K3 + (size_t)K2 * (K3 / 2 + 1));
}

bool plane_fwd_available(const qeq_plan* pl) {
    const KParams& k = pl->kp;
    if (!pl->fused_forward || k.K1 < 64 || k.p != 6) return false;
#define X(A, B) if (k.K2 == A && k.K3 == B) return true;
    QEQ_FOR_EACH_PLANE_FWD(X)
#undef X
    return false;
}

int plane_fwd_pass(qeq_plan* pl, const double* src, const int* done) {
    const KParams& k = pl->kp;
    ProfScope ps(pl, PK_SPREAD_R2C);
#define X(A, B)                                                                                    \
    if (k.K2 == A && k.K3 == B && k.p == 6) {                                                      \
        const size_t sh = smem_plane_fwd(A, B);                                                    \
        QEQ_HIP(hipFuncSetAttribute((const void*)k_plane_fwd<A, B>,                                \
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));         \
        hipExtLaunchKernelGGL((k_plane_fwd<A, B>), dim3(k.K1), dim3(PLANE_NT), sh, pl->stream, ps.start(), \
                              ps.stop(), 0, k, pl->axes.ax[1], pl->axes.ax[2], src, pl->bin_start, \
                              pl->home, pl->wts, pl->grid_c, done);                                 \
        return qeq_check(hipGetLastError());                                                       \
    }
    QEQ_FOR_EACH_PLANE_FWD(X)
#undef X
    return QEQ_EPLAN;
}

// Spread and forward axis-2 transform: the fused plane kernel where it
// applies, else the spread pass and the axis-2 pass.
int forward_head(qeq_plan* pl, const double* src, const int* done) {
    if (plane_fwd_available(pl)) return plane_fwd_pass(pl, src, done);
    QEQ_TRY(spread_pass(pl, src, done));
    return rows_pass(pl, 0, done);
}

// Inverse transforms after the axis-1 pass: the fused slab kernel where it
// applies, else the inverse axis-2 pass and the complex-to-real pass.
int inverse_tail(qeq_plan* pl, const int* done) {
    if (slab_available(pl)) return slab_inv_pass(pl, done);
    QEQ_TRY(rows_pass(pl, 1, done));
    return c2r_pass(pl, done);
}

}  // namespace

bool spread_tile_compiled(int K3, int tws, int p) {
#define X(KK, TT) if (K3 == KK && tws == TT && p == 6) return true;
    QEQ_FOR_EACH_SPREAD(X)
#undef X
    return false;
}

size_t qeq_mesh_max_smem(const KParams& k) {
    size_t a = smem_spread(k), b = smem_rows(k), c = smem_cols(k), d = smem_c2r(k);
    size_t m = a > b ? a : b;
    m = m > c ? m : c;
    return m > d ? m : d;
}

int launch_mesh_potential(qeq_plan* pl, const double* src, const int* done) {
    QEQ_TRY(forward_head(pl, src, done));
    QEQ_TRY(cols_pass(pl, MESH_FWD | MESH_GREEN | MESH_INV, nullptr, done));
    return inverse_tail(pl, done);
}

int launch_mesh_cg(qeq_plan* pl, const double* src, const int* done, bool* partials) {
    *partials = false;
    const bool slab = slab_interp_available(pl);
    if (!slab && !c2r_interp_available(pl)) return launch_mesh_potential(pl, src, done);
    QEQ_TRY(forward_head(pl, src, done));
    QEQ_TRY(cols_pass(pl, MESH_FWD | MESH_GREEN | MESH_INV, nullptr, done));
    *partials = true;
    if (slab) return slab_interp_pass(pl, done);
    QEQ_TRY(rows_pass(pl, 1, done));
    return c2r_interp_pass(pl, done);
}

int launch_mesh_from_spectrum(qeq_plan* pl, const int* done) {
    QEQ_TRY(rows_pass(pl, 0, done));
    QEQ_TRY(cols_pass(pl, MESH_FWD | MESH_GREEN | MESH_INV, nullptr, done));
    return inverse_tail(pl, done);
}

// One pass on its own (for timing): the spread, or the complex-to-real pass
// that the CG products run (interpolating from LDS where they do).
int launch_mesh_stage(qeq_plan* pl, int kind, const double* src) {
    if (kind == PK_SPREAD_R2C)
        return plane_fwd_available(pl) ? plane_fwd_pass(pl, src, nullptr) : spread_pass(pl, src, nullptr);
    if (kind == PK_C2R) {
        if (slab_interp_available(pl)) return slab_interp_pass(pl, nullptr);
        if (c2r_interp_available(pl)) return c2r_interp_pass(pl, nullptr);
        return slab_available(pl) ? slab_inv_pass(pl, nullptr) : c2r_pass(pl, nullptr);
    }
    return QEQ_EINVAL;
}

int launch_mesh_inverse(qeq_plan* pl) {
    QEQ_TRY(cols_pass(pl, MESH_INV, nullptr, nullptr));
    return inverse_tail(pl, nullptr);
}

int launch_write_green(qeq_plan* pl) {
    const KParams& k = pl->kp;
    const size_t total = (size_t)k.K3h * k.K1 * k.K2;
    hipLaunchKernelGGL(k_write_green, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, pl->stream, k,
                       pl->grid_c, pl->bmod[0], pl->bmod[1], pl->bmod[2]);
    return qeq_check(hipGetLastError());
}

int launch_write_green_strain(qeq_plan* pl, int comp) {
    const KParams& k = pl->kp;
    const size_t total = (size_t)k.K3h * k.K1 * k.K2;
    hipLaunchKernelGGL(k_write_green_strain, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, pl->stream, k,
                       pl->grid_c, pl->bmod[0], pl->bmod[1], pl->bmod[2], comp);
    return qeq_check(hipGetLastError());
}

int mesh_virial_blocks(const KParams& k) { return k.K3h * k.ntile; }

int launch_mesh_virial(qeq_plan* pl, const double* src, double* part) {
    QEQ_TRY(spread_pass(pl, src, nullptr));
    QEQ_TRY(rows_pass(pl, 0, nullptr));
    return cols_virial_pass(pl, part);
}
