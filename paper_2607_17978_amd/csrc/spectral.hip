// Spectral (k-space) preconditioner for the projected CG.
//
// The Electrostatics Solvers section notes that the CG iteration count grows
// with the system size; the growth comes from the long-wavelength Coulomb
// modes, whose eigenvalues (4 pi rho / k^2 at small k) a diagonal
// preconditioner cannot reach.  Their part of A is known exactly from the
// plane-wave form of the periodic Gaussian-charge energy:
//
//   sum_{k in a half space, |k| <= k_c} w_k (c_k c_k^T + s_k s_k^T),
//   w_k = 2 (4 pi / V) / k^2,  c_k,i = F_i(k) cos(k.r_i),  s_k,i = F_i(k) sin(k.r_i),
//   F_i(k) = exp(-sigma_i^2 k^2 / 2).
//
// With Phi = [c_k | s_k] (n x 2m columns, cosines first) and W = diag(w):
//   M = D' + Phi W Phi^T,  D' = D - diag(Phi W Phi^T)  (diag M = the Jacobi D),
//   M^-1 = D'^-1 - D'^-1 Phi S Phi^T D'^-1,  S = (W^-1 + Phi^T D'^-1 Phi)^-1,
// symmetric positive definite whenever D' > 0.  G = W^-1 + Phi^T D'^-1 Phi is
// diagonally dominant in practice (the spectrum of d G d, d = diag(G)^-1/2,
// lies around 1), so with E = I - d G d
//   S = d (I + E)(I + E^2)(I + E^4) ... d  (error E^(2^K) after K factors),
// two dense products of size 2m per factor.  The solution is unchanged: any
// SPD preconditioner of the projected CG converges to the same charges.
//
// The columns enter through one table per geometry, Psi = D'^-1/2 Phi rounded
// to BF16 (mode-major: row a holds column a for every atom).  The
// preconditioner is defined by that table, M = D'^1/2 (I + Psi W Psi^T) D'^1/2,
// so every piece below uses the same numbers and M stays exactly symmetric:
//   G = W^-1 + Psi^T Psi     BF16 MFMA, exact products, FP32 accumulation per
//                            atom split, FP64 over splits; upper tile pairs
//   M^-1 r = D'^-1/2 (u - Psi S Psi^T u),  u = D'^-1/2 r,
// two memory-bound passes over the table per iteration (t = Psi^T u over
// column groups x atom splits, then v = Psi s over atom blocks), with
// s = S t in between.  The search direction is then p = w - c M^-1 1 + beta p
// with c = sum(w) / sum(M^-1 1), keeping sum(p) = 0.
#include <math.h>

#include <algorithm>
#include <vector>

#include "internal.h"

namespace {

constexpr int SPC_MAX_MODES = 384;   // 768 columns
constexpr int SPC_T = 128;           // tile of the Gram matrix; dense matrices padded to it
constexpr int SPC_GSPLIT_MAX = 32;   // atom splits of the Gram matrix
constexpr int SPC_ATOM_PAD = 256;    // table rows padded to this many atoms
constexpr int SPC_FROWS = 16;        // table rows per block of t = Psi^T u (4 per wave)
constexpr int SPC_FSPLIT_MAX = 16;   // atom splits of t = Psi^T u
constexpr int SPC_KSPLIT = 4;        // k splits of the dense products
constexpr int SPC_BATOMS = 256;      // atoms per block of v = Psi s (four per lane)
constexpr double PI = 3.14159265358979323846;

// F_i(k) (cos, sin)(k.r_i) with k.r = 2 pi m.s (fractional coordinates), the
// argument reduced to one turn before the transcendental.
__device__ __forceinline__ void spc_phase(const float4 a, const int4 m, float k2, float& c, float& s) {
    float t = (float)m.x * a.x + (float)m.y * a.y + (float)m.z * a.z;
    t -= rintf(t);
    float sn, cs;
    sincospif(2.0f * t, &sn, &cs);
    const float f = __expf(-0.5f * a.w * k2);
    c = f * cs;
    s = f * sn;
}

typedef short spc_s4 __attribute__((ext_vector_type(4)));
typedef float spc_f4 __attribute__((ext_vector_type(4)));
typedef double spc_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short spc_bf16(float x) {   // round to nearest even
    unsigned u = __float_as_uint(x);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (unsigned short)((u >> 16) | 0x40u);   // NaN stays a (quiet) NaN
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float spc_f32(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// Per atom: compact coordinates and 1/D' with D' = D - sum_k w_k F_i(k)^2
// (cos^2 + sin^2 = 1); per block the largest fraction (D - D') / D.
__global__ void k_spc_atoms(int n, int nm, const double* __restrict__ frac, const double* __restrict__ sig,
                            const double* __restrict__ dinv, const float* __restrict__ k2,
                            const float* __restrict__ wk, float4* __restrict__ atom, double* __restrict__ dpinv,
                            float* __restrict__ sd, double* __restrict__ part) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double v[1] = {0.0};
    if (i < n) {
        const double s2 = sig[i] * sig[i];
        atom[i] = make_float4((float)frac[3 * i], (float)frac[3 * i + 1], (float)frac[3 * i + 2], (float)s2);
        double lr = 0.0;
        for (int m = 0; m < nm; ++m) lr += (double)wk[m] * exp(-s2 * (double)k2[m]);
        const double d = 1.0 / dinv[i];
        const double dp = d - lr;
        dpinv[i] = 1.0 / dp;
        sd[i] = (float)sqrt(1.0 / dp);
        v[0] = lr / d;   // fraction of the diagonal moved into the low-rank part
    }
    // block maximum of lr / D (reported through the partials as a max)
    __shared__ double mx[QEQ_BLOCK / 64];
    double x = v[0];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
    if ((threadIdx.x & 63) == 0) mx[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, mx[w]);
        part[blockIdx.x] = m;
    }
}

// Table rows: Psi[a][i] = bf16(D'_i^-1/2 (cos | sin)(k_m . r_i) F_i(k_m)),
// cosines in rows 0..nm-1, sines in nm..2nm-1; padded atoms and rows
// 2nm..ncp-1 are zero.  Block (atom block, group of 16 modes).
__global__ __launch_bounds__(256) void k_spc_psi(int n, int npad, int nm, int ncp, const int4* __restrict__ modes,
                                                 const float* __restrict__ k2, const float4* __restrict__ atom,
                                                 const float* __restrict__ sd, unsigned short* __restrict__ psi) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    const int m0 = blockIdx.y * 16;
    float4 a4 = make_float4(0.f, 0.f, 0.f, 0.f);
    float sc = 0.f;
    if (i < n) {
        a4 = atom[i];
        sc = sd[i];
    }
    for (int q = 0; q < 16; ++q) {
        const int m = m0 + q;
        if (m >= nm) break;
        float c = 0.f, sn = 0.f;
        if (i < n) spc_phase(a4, modes[m], k2[m], c, sn);
        psi[(size_t)m * npad + i] = spc_bf16(sc * c);
        psi[(size_t)(nm + m) * npad + i] = spc_bf16(sc * sn);
    }
    if (blockIdx.y == 0)
        for (int row = 2 * nm; row < ncp; ++row) psi[(size_t)row * npad + i] = 0;
}

// Split partial sums of Psi^T Psi over the upper tile pairs ta <= tb of
// SPC_T x SPC_T tiles.  Four waves per block, each a 64 x 64 quarter of the
// tile as 4 x 4 MFMA 16x16x16 bf16 accumulators.  The contraction runs over
// atoms in chunks of 32: lane l loads 8 consecutive atoms (16 bytes) of its
// row l%16 at atom offset 8 (l/16) and feeds them as two k-steps; A (rows a)
// and B (columns b) take the same atoms for the same k, so the sum covers
// every atom once.  Entries with a <= b are written to (a, b) and (b, a).
__global__ __launch_bounds__(256) void k_spc_gram(int npad, int ncp, int nt, int gsplit,
                                                  const unsigned short* __restrict__ psi,
                                                  float* __restrict__ gpart) {
    // one XCD holds consecutive logical blocks, i.e. all tile pairs of a few
    // atom splits, so each split's rows of the table are fetched into one L2
    const int ntp = nt * (nt + 1) / 2;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int sp = lb / ntp;
    // tile pair from the linear index: row ta holds pairs (ta, ta..nt-1)
    int t = lb - sp * ntp, ta = 0;
    while (t >= nt - ta) {
        t -= nt - ta;
        ++ta;
    }
    const int tb = ta + t;
    const int nch = npad / 32;
    const int per = (nch + gsplit - 1) / gsplit;
    const int c0 = sp * per, c1 = min(nch, c0 + per);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int arow = ta * SPC_T + 64 * (w >> 1), bcol = tb * SPC_T + 64 * (w & 1);
    const unsigned short* pa = psi + (size_t)(arow + r) * npad + 8 * g;
    const unsigned short* pb = psi + (size_t)(bcol + r) * npad + 8 * g;
    const size_t rs = (size_t)16 * npad;   // 16 rows on
    spc_f4 acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = spc_f4{0.f, 0.f, 0.f, 0.f};
    for (int c = c0; c < c1; ++c) {
        const size_t off = (size_t)c * 32;
        spc_s4 A[4][2], B[4][2];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const spc_s4* qa = (const spc_s4*)(pa + u * rs + off);
            const spc_s4* qb = (const spc_s4*)(pb + u * rs + off);
            A[u][0] = qa[0];
            A[u][1] = qa[1];
            B[u][0] = qb[0];
            B[u][1] = qb[1];
        }
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    acc[u][v] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[u][k], B[v][k], acc[u][v], 0, 0, 0);
    }
    // D layout: lane l holds rows 4 (l/16) + j of column l%16
    float* out = gpart + (size_t)sp * ncp * ncp;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int a = arow + 16 * u + 4 * g + j, b = bcol + 16 * v + r;
                if (a <= b) {
                    out[(size_t)a * ncp + b] = acc[u][v][j];
                    out[(size_t)b * ncp + a] = acc[u][v][j];
                }
            }
}

// The dense matrices below are ncp x ncp with zero rows and columns past nc.
// G = W^-1 + sum of the splits.
__global__ void k_spc_greduce(int nm, int ncp, int gsplit, const float* __restrict__ gpart,
                              const float* __restrict__ winv, double* __restrict__ G) {
    const int nc = 2 * nm;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)ncp * ncp) return;
    const int a = (int)(t / ncp), b = (int)(t - (size_t)a * ncp);
    double v = 0.0;
    if (a < nc && b < nc) {
        for (int sp = 0; sp < gsplit; ++sp) v += (double)gpart[(size_t)sp * ncp * ncp + t];
        if (a == b) v += (double)winv[a < nm ? a : a - nm];
    }
    G[t] = v;
}

// E = I - d G d, P = I + E; partial sums of ||E||_F^2 per block.
__global__ void k_spc_escale(int nc, int ncp, const double* __restrict__ G, double* __restrict__ E,
                             double* __restrict__ P, double* __restrict__ part) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v[1] = {0.0};
    if (t < (size_t)ncp * ncp) {
        const int a = (int)(t / ncp), b = (int)(t - (size_t)a * ncp);
        double e = 0.0, pv = 0.0;
        if (a < nc && b < nc) {
            e = (a == b ? 1.0 : 0.0) - G[t] / sqrt(G[(size_t)a * ncp + a] * G[(size_t)b * ncp + b]);
            pv = (a == b ? 1.0 : 0.0) + e;
        }
        E[t] = e;
        P[t] = pv;
        v[0] = e * e;
    }
    block_sum<1>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// Partial sums of squares of a dense matrix (its Frobenius norm).
__global__ void k_spc_sumsq(int ncp, const double* __restrict__ X, double* __restrict__ part) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v[1] = {0.0};
    if (t < (size_t)ncp * ncp) v[0] = X[t] * X[t];
    block_sum<1>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// Partial products C_z = A B over the k range z of SPC_KSPLIT, for symmetric
// A and B that commute (all are polynomials in E), FP64 MFMA 16x16x4.
// Symmetry lets both operands be read along rows: the A operand element
// (i, k) is A[k][i].  Four waves per block, each a 16 x 32 strip (two
// accumulators); block tile 32 x 64; grid.z = k split.
__global__ __launch_bounds__(256) void k_spc_gemm(int ncp, const double* __restrict__ A, const double* __restrict__ B,
                                                  double* __restrict__ Cpart) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int row0 = blockIdx.y * 32 + 16 * (w >> 1), col0 = blockIdx.x * 64 + 32 * (w & 1);
    const int kper = ncp / SPC_KSPLIT;
    const int kb = blockIdx.z * kper, ke = kb + kper;
    spc_d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k0 = kb; k0 < ke; k0 += 4) {
        const size_t kr = (size_t)(k0 + g) * ncp;
        const double a = A[kr + row0 + r];
        const double b0 = B[kr + col0 + r], b1 = B[kr + col0 + 16 + r];
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b1, acc1, 0, 0, 0);
    }
    // D layout: lane l holds rows 4 (l/16) + j of column l%16
    double* C = Cpart + (size_t)blockIdx.z * ncp * ncp;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const size_t o = (size_t)(row0 + 4 * g + j) * ncp + col0 + r;
        C[o] = acc0[j];
        C[o + 16] = acc1[j];
    }
}

// C = sum of the k-split partials (+ X if X is given).
__global__ void k_spc_gsum(int ncp, const double* __restrict__ Cpart, const double* __restrict__ X,
                           double* __restrict__ C) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t nn = (size_t)ncp * ncp;
    if (t >= nn) return;
    double v = X ? X[t] : 0.0;
#pragma unroll
    for (int z = 0; z < SPC_KSPLIT; ++z) v += Cpart[z * nn + t];
    C[t] = v;
}

// S = d P d (zero past nc).
__global__ void k_spc_sfinal(int nc, int ncp, const double* __restrict__ G, const double* __restrict__ P,
                             double* __restrict__ S) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)ncp * ncp) return;
    const int a = (int)(t / ncp), b = (int)(t - (size_t)a * ncp);
    S[t] = (a < nc && b < nc) ? P[t] / sqrt(G[(size_t)a * ncp + a] * G[(size_t)b * ncp + b]) : 0.0;
}

// u = D'^-1/2 r in FP32, zero on the padded atoms.
__global__ void k_spc_u(int n, int npad, const float* __restrict__ sd, const double* __restrict__ r,
                        float* __restrict__ u, const int* __restrict__ done) {
    if (done && *done) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npad) u[i] = i < n ? (float)((double)sd[i] * r[i]) : 0.f;
}

// t partials, t = Psi^T u: block (group of SPC_FROWS table rows, atom
// split); wave q takes rows 4q..4q+3 of the group, lane l atoms 4l..4l+3 of
// each 256-atom step (one 16-byte load of u, one 8-byte load per row), FP32
// products.  The 4 sums are reduced over the wave by a halving butterfly
// (the exchange over lane bit 5 hands over rows 2-3 or 0-1, the one over bit
// 4 the odd or even row) and then by plain exchanges; tpart[split][row].
__global__ __launch_bounds__(256) void k_spc_fwd(int npad, int ncp, int fsplit, const unsigned short* __restrict__ psi,
                                                 const float* __restrict__ u, double* __restrict__ tpart,
                                                 const int* __restrict__ done) {
    if (done && *done) return;
    // one XCD holds consecutive logical blocks: all row groups of a few atom
    // splits, which share the loads of u
    const int ng = ncp / SPC_FROWS;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int sp = lb / ng;
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int a0 = (lb - sp * ng) * SPC_FROWS + 4 * q;
    const int steps = npad / 256;
    const int per = (steps + fsplit - 1) / fsplit;
    const int s0 = sp * per, s1 = min(steps, s0 + per);
    const unsigned short* p = psi + (size_t)a0 * npad + 4 * lane;
    float v[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int st = s0; st < s1; ++st) {
        const int i = st * 256;
        const float4 uu = *(const float4*)(u + i + 4 * lane);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint2 h = *(const uint2*)(p + (size_t)c * npad + i);
            v[c] += uu.x * spc_f32((unsigned short)(h.x & 0xFFFFu)) + uu.y * spc_f32((unsigned short)(h.x >> 16)) +
                    uu.z * spc_f32((unsigned short)(h.y & 0xFFFFu)) + uu.w * spc_f32((unsigned short)(h.y >> 16));
        }
    }
    {   // bit 5: keep rows 0-1 (lower lanes) or 2-3 (upper lanes)
        const bool up = (lane & 32) != 0;
        const float s0v = up ? v[0] : v[2], s1v = up ? v[1] : v[3];
        const float k0 = up ? v[2] : v[0], k1 = up ? v[3] : v[1];
        v[0] = k0 + __shfl_xor(s0v, 32, 64);
        v[1] = k1 + __shfl_xor(s1v, 32, 64);
    }
    {   // bit 4: keep the even or the odd row
        const bool up = (lane & 16) != 0;
        const float sv = up ? v[0] : v[1], kv = up ? v[1] : v[0];
        v[0] = kv + __shfl_xor(sv, 16, 64);
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) v[0] += __shfl_xor(v[0], off, 64);
    // lane 16 b + ... holds row 2 (bit 5) + (bit 4)
    if ((lane & 15) == 0) tpart[(size_t)sp * ncp + a0 + 2 * ((lane >> 5) & 1) + ((lane >> 4) & 1)] = (double)v[0];
}

// t = sum of the split partials: one wave per row.
__global__ __launch_bounds__(256) void k_spc_treduce(int nc, int ncp, int fsplit, const double* __restrict__ tpart,
                                                     double* __restrict__ t, const int* __restrict__ done) {
    if (done && *done) return;
    const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= nc) return;   // whole waves
    double v = 0.0;
    for (int sp = lane; sp < fsplit; sp += 64) v += tpart[(size_t)sp * ncp + row];
    v = wave_sum(v);
    if (lane == 0) t[row] = v;
}

// s = S t: one wave per row, 16 rows per block.
__global__ __launch_bounds__(1024) void k_spc_mid(int nm, int ncp, const double* __restrict__ S,
                                                  const double* __restrict__ t, double* __restrict__ sout,
                                                  const int* __restrict__ done) {
    if (done && *done) return;
    extern __shared__ double tsh[];
    const int nc = 2 * nm;
    for (int a = threadIdx.x; a < nc; a += blockDim.x) tsh[a] = t[a];
    __syncthreads();
    const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= nc) return;   // whole waves
    double v = 0.0;
    for (int b = lane; b < nc; b += 64) v += S[(size_t)row * ncp + b] * tsh[b];
    v = wave_sum(v);
    if (lane == 0) sout[row] = v;
}

// w = D'^-1/2 (u - Psi s), u = D'^-1/2 r: block of SPC_BATOMS atoms, lane l
// takes atoms 4l .. 4l+3 (one 8-byte load per row), wave q the rows
// q ncp/4 .. (q+1) ncp/4 - 1, summed across the waves in LDS; partials
// [sum w, sum r w, sum r^2] per block.
__global__ __launch_bounds__(256) void k_spc_back(int n, int npad, int nm, int ncp,
                                                  const unsigned short* __restrict__ psi,
                                                  const float* __restrict__ sd, const double* __restrict__ r,
                                                  const double* __restrict__ s, double* __restrict__ w,
                                                  double* __restrict__ part, const int* __restrict__ done) {
    if (done && *done) return;
    __shared__ float ssh[2 * SPC_MAX_MODES + SPC_T];
    __shared__ float red[4][SPC_BATOMS];
    const int nc = 2 * nm;
    for (int a = threadIdx.x; a < ncp; a += blockDim.x) ssh[a] = a < nc ? (float)s[a] : 0.f;
    __syncthreads();
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int i = blockIdx.x * SPC_BATOMS + 4 * lane;
    const int rows = ncp / 4, a0 = q * rows;
    float v0 = 0.f, v1 = 0.f, v2 = 0.f, v3 = 0.f;
    if (i < npad) {
        // 8-byte loads (four atoms) and four rows in flight per lane
        const unsigned short* p = psi + (size_t)a0 * npad + i;
#pragma unroll 4
        for (int a = 0; a < rows; ++a) {
            const uint2 h = *(const uint2*)(p + (size_t)a * npad);
            const float sa = ssh[a0 + a];
            v0 += sa * spc_f32((unsigned short)(h.x & 0xFFFFu));
            v1 += sa * spc_f32((unsigned short)(h.x >> 16));
            v2 += sa * spc_f32((unsigned short)(h.y & 0xFFFFu));
            v3 += sa * spc_f32((unsigned short)(h.y >> 16));
        }
    }
    red[q][4 * lane] = v0;
    red[q][4 * lane + 1] = v1;
    red[q][4 * lane + 2] = v2;
    red[q][4 * lane + 3] = v3;
    __syncthreads();
    double pv[3] = {0.0, 0.0, 0.0};
    if (threadIdx.x < SPC_BATOMS) {
        const int ii = blockIdx.x * SPC_BATOMS + threadIdx.x;
        if (ii < n) {
            const float vv = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
            const double ri = r[ii], sdi = (double)sd[ii];
            const double wi = sdi * (sdi * ri - (double)vv);
            w[ii] = wi;
            pv[0] = wi;
            pv[1] = ri * wi;
            pv[2] = ri * ri;
        }
    }
    block_sum<3>(pv);
    if (threadIdx.x == 0)
        for (int t = 0; t < 3; ++t) part[(size_t)blockIdx.x * QEQ_NPART + t] = pv[t];
}

// sum(M^-1 1) from the partials of k_spc_back applied to the ones vector.
__global__ void k_spc_m1sum(const double* __restrict__ part, int nparts, const double* __restrict__ w,
                            double* __restrict__ m1, int n, double* __restrict__ scal) {
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) v[0] += part[(size_t)b * QEQ_NPART];
    block_sum<1>(v);
    if (threadIdx.x == 0) scal[0] = v[0];
    for (int i = threadIdx.x; i < n; i += blockDim.x) m1[i] = w[i];
}

// p = w - c M^-1 1 + beta p with c = sum(w) / sum(M^-1 1) (sum(p) stays 0),
// r.z = r.w - c sum(w); the relative residual decides convergence.
__global__ void k_spc_dir(KParams k, const double* __restrict__ w, const double* __restrict__ m1,
                          double* __restrict__ p, const double* __restrict__ part, int nparts,
                          const double* __restrict__ scal, CgScalars* sc, int parity, int init) {
    if (sc->done) return;
    __shared__ double tot[3];
    double v[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nparts; b += blockDim.x)
        for (int t = 0; t < 3; ++t) v[t] += part[(size_t)b * QEQ_NPART + t];
    block_sum<3>(v);
    if (threadIdx.x == 0)
        for (int t = 0; t < 3; ++t) tot[t] = v[t];
    __syncthreads();
    const double c = tot[0] / scal[0];
    const double rz = tot[1] - c * tot[0];
    const double beta = init ? 0.0 : rz / sc->rz[parity];
    const double res = sc->chi_norm > 0.0 ? sqrt(tot[2]) / sc->chi_norm : sqrt(tot[2]);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k.n) p[i] = w[i] - c * m1[i] + (init ? 0.0 : beta * p[i]);   // first direction: p not read
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->rz[parity ^ 1] = rz;
        sc->res = res;
        if (res <= k.tol || !(res == res)) sc->done = 1;
    }
}

__global__ void k_spc_fill(double* __restrict__ x, int n, double v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

template <typename T>
int spc_alloc(T** p, size_t count) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    if (hipMalloc((void**)p, sizeof(T) * (count ? count : 1)) != hipSuccess) return QEQ_ENOMEM;
    if (poisonable<T>) debug_poison(*p, sizeof(T) * count);
    return QEQ_OK;
}

double* part2(qeq_plan* pl) { return pl->part + (size_t)pl->nblk_max * QEQ_NPART; }

// Half-space modes with 0 < |k| <= k_c, k = 2 pi H^-1 m, nearest first.
void spc_modes(const KParams& k, double kc, std::vector<int>& mm, std::vector<float>& k2v) {
    struct Md { double k2; int m[3]; };
    std::vector<Md> all;
    int lim[3];
    for (int a = 0; a < 3; ++a) {
        const double len = sqrt(k.H[a * 3] * k.H[a * 3] + k.H[a * 3 + 1] * k.H[a * 3 + 1] +
                                k.H[a * 3 + 2] * k.H[a * 3 + 2]);
        lim[a] = (int)ceil(kc * len / (2 * PI)) + 1;
    }
    for (int m1 = 0; m1 <= lim[0]; ++m1)
        for (int m2 = -lim[1]; m2 <= lim[1]; ++m2)
            for (int m3 = -lim[2]; m3 <= lim[2]; ++m3) {
                // half space: first nonzero index positive
                if (m1 == 0 && (m2 < 0 || (m2 == 0 && m3 <= 0))) continue;
                double kv[3];
                for (int c = 0; c < 3; ++c)
                    kv[c] = 2 * PI * (k.Hinv[c * 3] * m1 + k.Hinv[c * 3 + 1] * m2 + k.Hinv[c * 3 + 2] * m3);
                const double q = kv[0] * kv[0] + kv[1] * kv[1] + kv[2] * kv[2];
                if (q <= kc * kc) all.push_back({q, {m1, m2, m3}});
            }
    std::sort(all.begin(), all.end(), [](const Md& a, const Md& b) { return a.k2 < b.k2; });
    if ((int)all.size() > SPC_MAX_MODES) all.resize(SPC_MAX_MODES);
    mm.clear();
    k2v.clear();
    for (const Md& d : all) {
        mm.push_back(d.m[0]);
        mm.push_back(d.m[1]);
        mm.push_back(d.m[2]);
        mm.push_back(0);
        k2v.push_back((float)d.k2);
    }
}

}  // namespace

void spc_free(qeq_plan* pl) {
    void* ptrs[] = {pl->spc_modes, pl->spc_k2, pl->spc_winv, pl->spc_wk, pl->spc_atom, pl->spc_dpinv,
                    pl->spc_sd, pl->spc_u, pl->spc_psi, pl->spc_mats, pl->spc_gpart, pl->spc_tpart, pl->spc_s,
                    pl->spc_wvec, pl->spc_m1, pl->spc_ones, pl->spc_scal, pl->spc_t, pl->spc_kpart};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    pl->spc_modes = nullptr;
    pl->spc_k2 = pl->spc_winv = pl->spc_wk = pl->spc_sd = pl->spc_u = pl->spc_gpart = nullptr;
    pl->spc_atom = nullptr;
    pl->spc_psi = nullptr;
    pl->spc_dpinv = pl->spc_mats = pl->spc_tpart = pl->spc_s = pl->spc_t = pl->spc_kpart = nullptr;
    pl->spc_wvec = pl->spc_m1 = pl->spc_ones = pl->spc_scal = nullptr;
    pl->spc_cap_m = pl->spc_cap_n = 0;
    pl->spc_active = false;
}

int spc_setup(qeq_plan* pl) {
    pl->spc_active = false;
    if (!(pl->spc_kc > 0.0)) return QEQ_OK;
    const KParams& k = pl->kp;
    std::vector<int> mm;
    std::vector<float> k2v;
    spc_modes(k, pl->spc_kc, mm, k2v);
    const int nm = (int)k2v.size();
    if (nm == 0) return QEQ_OK;   // no mode below the cutoff: Jacobi
    const int nc = 2 * nm;
    const int ncp = (nc + SPC_T - 1) / SPC_T * SPC_T;
    const size_t cmax = 2 * (size_t)SPC_MAX_MODES;
    const size_t epart = cmax * cmax / 256 + 1;   // blocks of the dense element-wise kernels (ncp <= cmax)
    if (!pl->spc_modes) {
        // mode tables and dense work space at the largest mode count, once
        QEQ_TRY(spc_alloc(&pl->spc_modes, (size_t)SPC_MAX_MODES));
        QEQ_TRY(spc_alloc(&pl->spc_k2, (size_t)SPC_MAX_MODES));
        QEQ_TRY(spc_alloc(&pl->spc_winv, (size_t)SPC_MAX_MODES));
        QEQ_TRY(spc_alloc(&pl->spc_wk, (size_t)SPC_MAX_MODES));
        QEQ_TRY(spc_alloc(&pl->spc_mats, 6 * cmax * cmax));
        QEQ_TRY(spc_alloc(&pl->spc_gpart, (size_t)SPC_GSPLIT_MAX * cmax * cmax));
        QEQ_TRY(spc_alloc(&pl->spc_s, cmax));
        QEQ_TRY(spc_alloc(&pl->spc_t, cmax));
        QEQ_TRY(spc_alloc(&pl->spc_kpart, (size_t)SPC_KSPLIT * cmax * cmax));
        pl->spc_cap_m = SPC_MAX_MODES;
    }
    const size_t nmat = (size_t)ncp * ncp;
    if (pl->spc_cap_n < pl->n_max) {
        const size_t n = (size_t)pl->n_max;
        const size_t np = (n + SPC_ATOM_PAD - 1) / SPC_ATOM_PAD * SPC_ATOM_PAD;
        const size_t fs = SPC_FSPLIT_MAX;
        QEQ_TRY(spc_alloc(&pl->spc_atom, n));
        QEQ_TRY(spc_alloc(&pl->spc_dpinv, n));
        QEQ_TRY(spc_alloc(&pl->spc_sd, n));
        QEQ_TRY(spc_alloc(&pl->spc_u, np));
        QEQ_TRY(spc_alloc(&pl->spc_psi, cmax * np));
        QEQ_TRY(spc_alloc(&pl->spc_tpart, std::max(fs * cmax, epart)));
        QEQ_TRY(spc_alloc(&pl->spc_wvec, n));
        QEQ_TRY(spc_alloc(&pl->spc_m1, n));
        QEQ_TRY(spc_alloc(&pl->spc_ones, n));
        QEQ_TRY(spc_alloc(&pl->spc_scal, 4));
        pl->spc_cap_n = pl->n_max;
    }
    const int n = k.n;
    const int npad = (n + SPC_ATOM_PAD - 1) / SPC_ATOM_PAD * SPC_ATOM_PAD;
    pl->spc_nm = nm;
    pl->spc_ncp = ncp;
    pl->spc_npad = npad;
    pl->spc_fsplit = std::min(SPC_FSPLIT_MAX, npad / 256);
    std::vector<float> winv(nm), wk(nm);
    for (int m = 0; m < nm; ++m) {
        const double w = 2.0 * 4.0 * PI / k.vol / (double)k2v[m];
        wk[m] = (float)w;
        winv[m] = (float)(1.0 / w);
    }
    QEQ_HIP(hipMemcpyAsync(pl->spc_modes, mm.data(), sizeof(int4) * nm, hipMemcpyHostToDevice, pl->stream));
    QEQ_HIP(hipMemcpyAsync(pl->spc_k2, k2v.data(), sizeof(float) * nm, hipMemcpyHostToDevice, pl->stream));
    QEQ_HIP(hipMemcpyAsync(pl->spc_winv, winv.data(), sizeof(float) * nm, hipMemcpyHostToDevice, pl->stream));
    QEQ_HIP(hipMemcpyAsync(pl->spc_wk, wk.data(), sizeof(float) * nm, hipMemcpyHostToDevice, pl->stream));
    const int nb = nblocks(n);
    double* pp = part2(pl);
    hipLaunchKernelGGL(k_spc_atoms, dim3(nb), dim3(QEQ_BLOCK), 0, pl->stream, n, nm, pl->frac, pl->sig, pl->dinv,
                       pl->spc_k2, pl->spc_wk, pl->spc_atom, pl->spc_dpinv, pl->spc_sd, pp);
    hipLaunchKernelGGL(k_spc_psi, dim3(npad / 256, (nm + 15) / 16), dim3(256), 0, pl->stream, n, npad, nm, ncp,
                       pl->spc_modes, pl->spc_k2, pl->spc_atom, pl->spc_sd, pl->spc_psi);
    QEQ_HIP(hipGetLastError());
    double* G = pl->spc_mats;
    double* E = G + nmat;
    double* E2 = E + nmat;
    double* P = E2 + nmat;
    double* Q = P + nmat;
    double* S = Q + nmat;
    // Gram over the upper tile pairs, about a thousand blocks in all
    const int ntg = ncp / SPC_T, ntp = ntg * (ntg + 1) / 2;
    const int nch = npad / 32;
    const int gsplit = std::max(1, std::min({SPC_GSPLIT_MAX, (1024 + ntp - 1) / ntp, nch}));
    hipLaunchKernelGGL(k_spc_gram, dim3(ntp * gsplit), dim3(256), 0, pl->stream, npad, ncp, ntg, gsplit,
                       (const unsigned short*)pl->spc_psi, pl->spc_gpart);
    const int eb = (int)((nmat + 255) / 256);
    hipLaunchKernelGGL(k_spc_greduce, dim3(eb), dim3(256), 0, pl->stream, nm, ncp, gsplit,
                       (const float*)pl->spc_gpart, pl->spc_winv, G);
    // ||E||_F^2 partials in the forward product's partial buffer, unused
    // until the first application
    double* pe = pl->spc_tpart;
    hipLaunchKernelGGL(k_spc_escale, dim3(eb), dim3(256), 0, pl->stream, nc, ncp, G, E, P, pe);
    QEQ_HIP(hipGetLastError());
    // checks on the host: D' > 0 with margin; the product series below
    // converges when the spectral radius of E is below 1
    std::vector<double> hp((size_t)nb + eb);
    QEQ_HIP(hipMemcpyAsync(hp.data(), pp, sizeof(double) * nb, hipMemcpyDeviceToHost, pl->stream));
    QEQ_HIP(hipMemcpyAsync(hp.data() + nb, pe, sizeof(double) * eb, hipMemcpyDeviceToHost, pl->stream));
    QEQ_HIP(hipStreamSynchronize(pl->stream));
    double lrmax = 0.0, e2 = 0.0;
    for (int b = 0; b < nb; ++b) lrmax = std::max(lrmax, hp[b]);
    for (int b = 0; b < eb; ++b) e2 += hp[(size_t)nb + b];
    const double en = sqrt(e2);
    if (!(lrmax < 0.9) || !(en == en)) return QEQ_OK;   // D' too small: keep Jacobi
    // (I - E)^-1 = (I + E)(I + E^2)(I + E^4)...; after the factors up to
    // E^(2^(j-1)) the error of the product is exactly E^(2^j).  With
    // ||E||_F < 0.9 the factor count follows from ||E^k||_F <= ||E||_F^k;
    // otherwise (small cells, where ||E||_F overstates the spectral radius)
    // the norm of each new power is read back until it falls below 1e-7, and
    // a power that does not shrink within 11 squarings means Jacobi.
    const bool bound = en < 0.9;
    int K = 1;
    if (bound)
        while (K < 12 && std::pow(std::max(en, 1e-300), (double)(1 << K)) > 1e-7) ++K;
    const dim3 gg(ncp / 64, ncp / 32, SPC_KSPLIT);
    double* kp = pl->spc_kpart;
    double* X = E;
    double* Xn = E2;
    for (int j = 1; bound ? j < K : true; ++j) {
        hipLaunchKernelGGL(k_spc_gemm, gg, dim3(256), 0, pl->stream, ncp, X, X, kp);   // E^(2^j)
        hipLaunchKernelGGL(k_spc_gsum, dim3(eb), dim3(256), 0, pl->stream, ncp, kp, (const double*)nullptr, Xn);
        if (!bound) {
            hipLaunchKernelGGL(k_spc_sumsq, dim3(eb), dim3(256), 0, pl->stream, ncp, Xn, pe);
            QEQ_HIP(hipMemcpyAsync(hp.data(), pe, sizeof(double) * eb, hipMemcpyDeviceToHost, pl->stream));
            QEQ_HIP(hipStreamSynchronize(pl->stream));
            double x2 = 0.0;
            for (int b = 0; b < eb; ++b) x2 += hp[b];
            if (sqrt(x2) <= 1e-7) break;                       // P is accurate to 1e-7
            if (!(sqrt(x2) < 1e6) || j >= 11) return QEQ_OK;   // not converging: Jacobi
        }
        hipLaunchKernelGGL(k_spc_gemm, gg, dim3(256), 0, pl->stream, ncp, P, Xn, kp);   // P (I + E^(2^j))
        hipLaunchKernelGGL(k_spc_gsum, dim3(eb), dim3(256), 0, pl->stream, ncp, kp, (const double*)P, Q);
        std::swap(X, Xn);
        std::swap(P, Q);
    }
    hipLaunchKernelGGL(k_spc_sfinal, dim3(eb), dim3(256), 0, pl->stream, nc, ncp, G, P, S);
    QEQ_HIP(hipGetLastError());
    // M^-1 1 and its sum
    hipLaunchKernelGGL(k_spc_fill, dim3(nb), dim3(QEQ_BLOCK), 0, pl->stream, pl->spc_ones, n, 1.0);
    pl->spc_active = true;
    QEQ_TRY(spc_apply(pl, pl->spc_ones, nullptr));
    hipLaunchKernelGGL(k_spc_m1sum, dim3(1), dim3(1024), 0, pl->stream, pp, npad / SPC_BATOMS, pl->spc_wvec,
                       pl->spc_m1, n, pl->spc_scal);
    return qeq_check(hipGetLastError());
}

int spc_apply(qeq_plan* pl, const double* r, const int* done, bool u_ready) {
    const KParams& k = pl->kp;
    const int nm = pl->spc_nm, nc = 2 * nm, ncp = pl->spc_ncp, npad = pl->spc_npad;
    const double* S = pl->spc_mats + 5 * (size_t)ncp * ncp;
    const unsigned short* psi = pl->spc_psi;
    if (!u_ready)
        hipLaunchKernelGGL(k_spc_u, dim3(npad / 256), dim3(256), 0, pl->stream, k.n, npad, pl->spc_sd, r, pl->spc_u,
                           done);
    hipLaunchKernelGGL(k_spc_fwd, dim3(ncp / SPC_FROWS * pl->spc_fsplit), dim3(256), 0, pl->stream, npad, ncp,
                       pl->spc_fsplit, psi, pl->spc_u, pl->spc_tpart, done);
    hipLaunchKernelGGL(k_spc_treduce, dim3((nc + 3) / 4), dim3(256), 0, pl->stream, nc, ncp, pl->spc_fsplit,
                       pl->spc_tpart, pl->spc_t, done);
    hipLaunchKernelGGL(k_spc_mid, dim3((nc + 15) / 16), dim3(1024), sizeof(double) * nc, pl->stream, nm, ncp, S,
                       pl->spc_t, pl->spc_s, done);
    hipLaunchKernelGGL(k_spc_back, dim3(npad / SPC_BATOMS), dim3(256), 0, pl->stream, k.n, npad, nm, ncp, psi,
                       pl->spc_sd, r, pl->spc_s, pl->spc_wvec, part2(pl), done);
    return qeq_check(hipGetLastError());
}

int spc_direction(qeq_plan* pl, int parity, int init) {
    const int nb = nblocks(pl->kp.n);
    hipLaunchKernelGGL(k_spc_dir, dim3(nb), dim3(QEQ_BLOCK), 0, pl->stream, pl->kp, pl->spc_wvec, pl->spc_m1,
                       pl->pvec, part2(pl), pl->spc_npad / SPC_BATOMS, pl->spc_scal, pl->sc, parity, init);
    return qeq_check(hipGetLastError());
}
