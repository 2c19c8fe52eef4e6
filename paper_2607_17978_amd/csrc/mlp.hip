// Learned warm start: radial descriptors from the QEq pair list and the
// per-element 16-32-32-1 tanh network (inference and training) on BF16 MFMA
// with FP32 accumulation.
//
// Descriptors (paper eq. g2 with the SI cosine cutoff): for every atom i,
//   G_i,mu = sum_j exp(-eta (r_ij - c_mu)^2) (cos(pi r_ij / r_c) + 1) / 2,  r_ij < r_c,
// over the image-aware pair list the solve already built.
//
// Network (SI feed-forward networks, tanh activations, linear output, one
// network per element), parameters per element packed as
//   W1 (32x16) | b1 (32) | W2 (32x32) | b2 (32) | W3 (32) | b3 (1), stride 1664 floats.
// Inputs are scaled per element as (G - mean) / (max - min) (SI feature scaling).
//
// MFMA mapping (v_mfma_f32_16x16x16 bf16, wave64): weights are the A operand
// (rows = output neurons, k = inputs), activations the B operand (k = inputs,
// columns = 16 atoms).  The D layout of one layer (lane l holds rows
// 4(l/16)+j of column l%16) is exactly the B layout the next layer needs, so
// the forward pass chains MFMAs in registers; the weight gradients, which
// contract over atoms, take their operands through small per-wave LDS
// transposes.
#include <math.h>

#include <mutex>

#include "internal.h"

namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

#define MLP_STRIDE 1664
#define MLP_W1 0
#define MLP_B1 512
#define MLP_W2 544
#define MLP_B2 1568
#define MLP_W3 1600
#define MLP_B3 1632
#define MLP_NF 16
#define MLP_MAXSP 4
#define MLP_BLOCKS 256          // blocks of the training kernel (partial gradients)
#define MLP_CLIP 1.5f           // scaled features are clipped to [-1.5, 1.5]

__device__ __forceinline__ short f2bf(float x) {   // round to nearest even
    unsigned u = __float_as_uint(x);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (short)((u >> 16) | 0x40u);   // NaN stays a (quiet) NaN
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

__device__ __forceinline__ f4 mfma(s4 a, s4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------ descriptors
struct DescParams {
    int nf;
    float centers[32];
    float eta;      // 1 / (2 width^2)
    float rc;
};

// G_i,mu = sum_j w_j exp(-eta (r_ij - c_mu)^2) f_c(r_ij) over the pair list
// (sorted order); w_j = weights[perm[j]] (caller order) or 1 without weights.
// Sixteen lanes per atom take its pair row in interleaved strides (the pair
// data of a row is contiguous, so the group's loads coalesce), each keeping
// partial sums of the nf functions; the sums are then reduced across the
// group and lane m writes feature m.
constexpr int DESC_G = 16;
__global__ __launch_bounds__(QEQ_BLOCK) void k_descriptors(int n, DescParams d, const int* __restrict__ rowptr,
                                                           const int* __restrict__ col,
                                                           const float4* __restrict__ pdr,
                                                           const int* __restrict__ perm,
                                                           const double* __restrict__ weights,
                                                           float* __restrict__ G) {
    const int lane = threadIdx.x & (DESC_G - 1);
    const int i = (blockIdx.x * blockDim.x + threadIdx.x) / DESC_G;
    if (i >= n) return;   // whole groups
    float acc[32];
#pragma unroll
    for (int m = 0; m < 32; ++m) acc[m] = 0.f;
    const float pi_rc = 3.14159265358979323846f / d.rc;
    const int e1 = rowptr[i + 1];
    for (int e = rowptr[i] + lane; e < e1; e += DESC_G) {
        const float4 v = pdr[e];
        const float r = sqrtf(v.x * v.x + v.y * v.y + v.z * v.z);
        if (r >= d.rc) continue;
        float fc = 0.5f * (cosf(pi_rc * r) + 1.f);
        if (weights) fc *= (float)weights[perm[col[e]]];
#pragma unroll
        for (int m = 0; m < 32; ++m) {
            if (m < d.nf) {
                const float t = r - d.centers[m];
                acc[m] += expf(-d.eta * t * t) * fc;
            }
        }
    }
    float* out = G + (size_t)perm[i] * d.nf;
#pragma unroll
    for (int m = 0; m < 32; ++m) {
        if (m < d.nf) {
            float a = acc[m];
#pragma unroll
            for (int off = DESC_G / 2; off > 0; off >>= 1) a += __shfl_xor(a, off, DESC_G);
            if (lane == (m & (DESC_G - 1))) out[m] = a;
        }
    }
}

// ------------------------------------------------------------------ feature statistics
// stats[s][0][f] = mean, [1][f] = min, [2][f] = max over the atoms of element s.
// Block = 16 atom slots x 16 features; each thread keeps per-element sum / min /
// max / count of its feature over its atoms, then the 16 slots are combined.
__global__ void k_feat_partial(const float* __restrict__ G, const int* __restrict__ species, int n, int nsp,
                               float* __restrict__ part) {
    __shared__ float sh[16][MLP_MAXSP][4];
    const int tid = threadIdx.x;
    const int f = tid & (MLP_NF - 1), slot = tid >> 4;
    float sum[MLP_MAXSP], mn[MLP_MAXSP], mx[MLP_MAXSP], cnt[MLP_MAXSP];
    for (int s = 0; s < MLP_MAXSP; ++s) {
        sum[s] = 0.f;
        mn[s] = 3.0e38f;
        mx[s] = -3.0e38f;
        cnt[s] = 0.f;
    }
    for (int a = blockIdx.x * 16 + slot; a < n; a += gridDim.x * 16) {
        const int s = species[a];
        const float g = G[(size_t)a * MLP_NF + f];
        for (int e = 0; e < MLP_MAXSP; ++e) {
            if (e != s) continue;
            sum[e] += g;
            mn[e] = fminf(mn[e], g);
            mx[e] = fmaxf(mx[e], g);
            cnt[e] += 1.f;
        }
    }
    float* o = part + (size_t)blockIdx.x * (MLP_MAXSP * (MLP_NF * 3 + 1));
    // combine the 16 slots through LDS, one feature per pass
    for (int ff = 0; ff < MLP_NF; ++ff) {
        __syncthreads();
        if (f == ff) {
            for (int s = 0; s < nsp; ++s) {
                sh[slot][s][0] = sum[s];
                sh[slot][s][1] = mn[s];
                sh[slot][s][2] = mx[s];
                sh[slot][s][3] = cnt[s];
            }
        }
        __syncthreads();
        if (tid < nsp) {
            const int s = tid;
            float a0 = 0.f, a1 = 3.0e38f, a2 = -3.0e38f, a3 = 0.f;
            for (int k = 0; k < 16; ++k) {
                a0 += sh[k][s][0];
                a1 = fminf(a1, sh[k][s][1]);
                a2 = fmaxf(a2, sh[k][s][2]);
                a3 += sh[k][s][3];
            }
            o[(s * MLP_NF + ff) * 3 + 0] = a0;
            o[(s * MLP_NF + ff) * 3 + 1] = a1;
            o[(s * MLP_NF + ff) * 3 + 2] = a2;
            if (ff == 0) o[MLP_MAXSP * MLP_NF * 3 + s] = a3;
        }
    }
}

__global__ void k_feat_finish(const float* __restrict__ part, int nblk, int nsp, float* __restrict__ stats) {
    const int t = threadIdx.x;   // one thread per (s, f)
    if (t >= nsp * MLP_NF) return;
    const int s = t / MLP_NF, f = t % MLP_NF;
    double sum = 0.0, cnt = 0.0;
    float mn = 3.0e38f, mx = -3.0e38f;
    const int stride = MLP_MAXSP * (MLP_NF * 3 + 1);
    for (int b = 0; b < nblk; ++b) {
        const float* o = part + (size_t)b * stride;
        sum += o[(s * MLP_NF + f) * 3 + 0];
        mn = fminf(mn, o[(s * MLP_NF + f) * 3 + 1]);
        mx = fmaxf(mx, o[(s * MLP_NF + f) * 3 + 2]);
        cnt += o[MLP_MAXSP * MLP_NF * 3 + s];
    }
    stats[(s * 3 + 0) * MLP_NF + f] = cnt > 0 ? (float)(sum / cnt) : 0.f;
    stats[(s * 3 + 1) * MLP_NF + f] = cnt > 0 ? mn : 0.f;
    stats[(s * 3 + 2) * MLP_NF + f] = cnt > 0 ? mx : 1.f;
}

// ------------------------------------------------------------------ network
struct NetRegs {
    s4 A1[2];        // W1 rows 16t + c, cols 4g + j
    s4 A2[2][2];     // W2 [u][t]: rows 16u + c, cols 16t + 4g + j
    s4 A2T[2][2];    // W2^T [t][u]: rows 16t + c, cols 16u + 4g + j
    float b1[2][4], b2[2][4], w3[2][4], b3;
    float mean[4], inv_rng[4];   // scaling of inputs 4g + j
};

__device__ __forceinline__ void load_net(NetRegs& R, const float* __restrict__ P, const float* __restrict__ st,
                                         int c, int g) {
    for (int t = 0; t < 2; ++t)
        for (int j = 0; j < 4; ++j) R.A1[t][j] = f2bf(P[MLP_W1 + (16 * t + c) * 16 + 4 * g + j]);
    for (int u = 0; u < 2; ++u)
        for (int t = 0; t < 2; ++t)
            for (int j = 0; j < 4; ++j) {
                R.A2[u][t][j] = f2bf(P[MLP_W2 + (16 * u + c) * 32 + 16 * t + 4 * g + j]);
                R.A2T[t][u][j] = f2bf(P[MLP_W2 + (16 * u + 4 * g + j) * 32 + 16 * t + c]);
            }
    for (int t = 0; t < 2; ++t)
        for (int j = 0; j < 4; ++j) {
            R.b1[t][j] = P[MLP_B1 + 16 * t + 4 * g + j];
            R.b2[t][j] = P[MLP_B2 + 16 * t + 4 * g + j];
            R.w3[t][j] = P[MLP_W3 + 16 * t + 4 * g + j];
        }
    R.b3 = P[MLP_B3];
    for (int j = 0; j < 4; ++j) {
        const int f = 4 * g + j;
        const float mn = st[1 * MLP_NF + f], mx = st[2 * MLP_NF + f];
        R.mean[j] = st[f];
        R.inv_rng[j] = (mx - mn) > 0.f ? 1.f / (mx - mn) : 1.f;
    }
}

// Training / inference kernel.  Block = 4 waves; every wave takes tiles of 16
// atoms; the number of rounds is uniform over the block so that block-wide
// barriers around the LDS transposes are safe.
template <bool TRAIN>
__global__ __launch_bounds__(256) void k_mlp(const float* __restrict__ G, const int* __restrict__ species,
                                            const double* __restrict__ target, int n, int nsp,
                                            const float* __restrict__ params, const float* __restrict__ stats,
                                            double* __restrict__ out, float* __restrict__ gpart,
                                            double* __restrict__ lpart, float inv_n) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int c = lane & 15, g = lane >> 4;
    __shared__ short tr[4][7][256];                  // per-wave transposes
    __shared__ float gs[TRAIN ? MLP_MAXSP * MLP_STRIDE : 1];
    if (TRAIN) {
        for (int t = tid; t < nsp * MLP_STRIDE; t += 256) gs[t] = 0.f;
        __syncthreads();
    }
    const int ntiles = (n + 15) / 16;
    const int rounds = (ntiles + 4 * gridDim.x - 1) / (4 * gridDim.x);
    double loss = 0.0;
    for (int sp = 0; sp < nsp; ++sp) {
        NetRegs R;
        load_net(R, params + (size_t)sp * MLP_STRIDE, stats + (size_t)sp * 3 * MLP_NF, c, g);
        f4 dW1[2], dW2[2][2];
        float db1[2][4], db2[2][4], dw3[2][4], db3 = 0.f;
        for (int t = 0; t < 2; ++t) {
            dW1[t] = f4{0.f, 0.f, 0.f, 0.f};
            for (int u = 0; u < 2; ++u) dW2[t][u] = f4{0.f, 0.f, 0.f, 0.f};
            for (int j = 0; j < 4; ++j) db1[t][j] = db2[t][j] = dw3[t][j] = 0.f;
        }
        for (int rnd = 0; rnd < rounds; ++rnd) {
            const int tile = (rnd * gridDim.x + blockIdx.x) * 4 + wv;
            const int a = tile * 16 + c;
            const bool mine = a < n && species[a] == sp;
            // B operand: scaled features 4g + j of atom a
            s4 xb;
            float4 gv = mine ? *reinterpret_cast<const float4*>(G + (size_t)a * MLP_NF + 4 * g)
                             : make_float4(0.f, 0.f, 0.f, 0.f);
            const float gx[4] = {gv.x, gv.y, gv.z, gv.w};
            // extrapolation guard: scaled features outside the training range are clipped
            for (int j = 0; j < 4; ++j)
                xb[j] = mine ? f2bf(fminf(fmaxf((gx[j] - R.mean[j]) * R.inv_rng[j], -MLP_CLIP), MLP_CLIP))
                             : (short)0;
            // layer 1
            float h1[2][4];
            s4 hb1[2];
            for (int t = 0; t < 2; ++t) {
                f4 z = mfma(R.A1[t], xb, f4{0.f, 0.f, 0.f, 0.f});
                for (int j = 0; j < 4; ++j) {
                    h1[t][j] = tanhf(z[j] + R.b1[t][j]);
                    hb1[t][j] = f2bf(h1[t][j]);
                }
            }
            // layer 2
            float h2[2][4];
            for (int u = 0; u < 2; ++u) {
                f4 z = mfma(R.A2[u][0], hb1[0], f4{0.f, 0.f, 0.f, 0.f});
                z = mfma(R.A2[u][1], hb1[1], z);
                for (int j = 0; j < 4; ++j) h2[u][j] = tanhf(z[j] + R.b2[u][j]);
            }
            // layer 3 (FP32): sum over the 32 hidden units held by the four lane groups
            float yp = 0.f;
            for (int u = 0; u < 2; ++u)
                for (int j = 0; j < 4; ++j) yp += R.w3[u][j] * h2[u][j];
            yp += __shfl_xor(yp, 16, 64);
            yp += __shfl_xor(yp, 32, 64);
            const float y = yp + R.b3;
            if (!TRAIN) {
                if (mine && g == 0) out[a] = (double)y;
                continue;
            }
            const float tgt = mine ? (float)target[a] : 0.f;
            const float dy = mine ? (y - tgt) * inv_n : 0.f;
            if (mine && g == 0) loss += 0.5 * (double)(y - tgt) * (double)(y - tgt) * (double)inv_n;
            if (g == 0) db3 += dy;
            float dz2[2][4];
            s4 dzb2[2];
            for (int u = 0; u < 2; ++u)
                for (int j = 0; j < 4; ++j) {
                    dw3[u][j] += dy * h2[u][j];
                    dz2[u][j] = dy * R.w3[u][j] * (1.f - h2[u][j] * h2[u][j]);
                    db2[u][j] += dz2[u][j];
                    dzb2[u][j] = f2bf(dz2[u][j]);
                }
            // dh1 = W2^T dz2 (dz2 in D layout is the B layout)
            s4 dzb1[2];
            for (int t = 0; t < 2; ++t) {
                f4 z = mfma(R.A2T[t][0], dzb2[0], f4{0.f, 0.f, 0.f, 0.f});
                z = mfma(R.A2T[t][1], dzb2[1], z);
                for (int j = 0; j < 4; ++j) {
                    const float d1 = z[j] * (1.f - h1[t][j] * h1[t][j]);
                    db1[t][j] += d1;
                    dzb1[t][j] = f2bf(d1);
                }
            }
            // transposes: value at (row 4g + j, column c) -> tr[.][(4g + j) * 16 + c]
            short* T = &tr[wv][0][0];
            for (int j = 0; j < 4; ++j) {
                const int o = (4 * g + j) * 16 + c;
                T[0 * 256 + o] = dzb2[0][j];
                T[1 * 256 + o] = dzb2[1][j];
                T[2 * 256 + o] = hb1[0][j];
                T[3 * 256 + o] = hb1[1][j];
                T[4 * 256 + o] = dzb1[0][j];
                T[5 * 256 + o] = dzb1[1][j];
                T[6 * 256 + o] = xb[j];
            }
            __syncthreads();
            // transposed reads: operand[(row c)][(k 4g + j)] = value(row c, column 4g + j)
            s4 tz2[2], th1[2], tz1[2], tx;
            for (int j = 0; j < 4; ++j) {
                const int o = c * 16 + 4 * g + j;
                tz2[0][j] = T[0 * 256 + o];
                tz2[1][j] = T[1 * 256 + o];
                th1[0][j] = T[2 * 256 + o];
                th1[1][j] = T[3 * 256 + o];
                tz1[0][j] = T[4 * 256 + o];
                tz1[1][j] = T[5 * 256 + o];
                tx[j] = T[6 * 256 + o];
            }
            __syncthreads();
            // dW2[u][t] = dz2_u (16 x atoms) . h1_t^T (atoms x 16)
            for (int u = 0; u < 2; ++u)
                for (int t = 0; t < 2; ++t) dW2[u][t] = mfma(tz2[u], th1[t], dW2[u][t]);
            // dW1[t] = dz1_t (16 x atoms) . X (atoms x 16 features)
            for (int t = 0; t < 2; ++t) dW1[t] = mfma(tz1[t], tx, dW1[t]);
        }
        if (!TRAIN) continue;
        // fold this wave's gradients into the block's LDS accumulator
        float* gsp = gs + sp * MLP_STRIDE;
        for (int t = 0; t < 2; ++t)
            for (int j = 0; j < 4; ++j) {
                atomicAdd(&gsp[MLP_W1 + (16 * t + 4 * g + j) * 16 + c], dW1[t][j]);
                for (int u = 0; u < 2; ++u)
                    atomicAdd(&gsp[MLP_W2 + (16 * u + 4 * g + j) * 32 + 16 * t + c], dW2[u][t][j]);
            }
        // per-lane vectors hold one atom column each: sum the 16 columns of a lane group
        for (int t = 0; t < 2; ++t)
            for (int j = 0; j < 4; ++j) {
                float v1 = db1[t][j], v2 = db2[t][j], v3 = dw3[t][j];
                for (int off = 1; off < 16; off <<= 1) {
                    v1 += __shfl_xor(v1, off, 64);
                    v2 += __shfl_xor(v2, off, 64);
                    v3 += __shfl_xor(v3, off, 64);
                }
                if (c == 0) {
                    atomicAdd(&gsp[MLP_B1 + 16 * t + 4 * g + j], v1);
                    atomicAdd(&gsp[MLP_B2 + 16 * t + 4 * g + j], v2);
                    atomicAdd(&gsp[MLP_W3 + 16 * t + 4 * g + j], v3);
                }
            }
        for (int off = 1; off < 64; off <<= 1) db3 += __shfl_xor(db3, off, 64);
        if (lane == 0) atomicAdd(&gsp[MLP_B3], db3);
    }
    if (TRAIN) {
        double lv[1] = {loss};
        block_sum<1>(lv);
        __syncthreads();
        float* o = gpart + (size_t)blockIdx.x * nsp * MLP_STRIDE;
        for (int t = tid; t < nsp * MLP_STRIDE; t += 256) o[t] = gs[t];
        if (tid == 0) lpart[blockIdx.x] = lv[0];
    }
}

__global__ void k_grad_reduce(const float* __restrict__ gpart, int nblk, int np, float* __restrict__ grad,
                              const double* __restrict__ lpart, float* __restrict__ loss) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < np) {
        float s = 0.f;
        for (int b = 0; b < nblk; ++b) s += gpart[(size_t)b * np + t];
        grad[t] = s;
    }
    if (t == 0 && loss) {
        double l = 0.0;
        for (int b = 0; b < nblk; ++b) l += lpart[b];
        *loss = (float)l;
    }
}

// Adam (SI: beta1 0.9, beta2 0.999, eps 1e-8); step counts from 1.  Padding
// entries of the packed layout stay zero.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ grad, float* __restrict__ m,
                       float* __restrict__ v, int np, int step, float lr) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= np) return;
    if (t % MLP_STRIDE > MLP_B3) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float gr = grad[t];
    const float mt = b1 * m[t] + (1.f - b1) * gr;
    const float vt = b2 * v[t] + (1.f - b2) * gr * gr;
    m[t] = mt;
    v[t] = vt;
    const float mh = mt / (1.f - powf(b1, (float)step));
    const float vh = vt / (1.f - powf(b2, (float)step));
    p[t] -= lr * mh / (sqrtf(vh) + eps);
}

// Workspace of mlp_train_step_noalloc: one fixed array per device (each GPU
// that runs it holds its own copy until the process ends), large enough for
// the largest n_species the kernels take.  Host code never uses the array's
// name as a pointer: it uses the device address hipGetSymbolAddress gives.
constexpr int64_t MLP_SCRATCH_FLOATS =
    (int64_t)MLP_BLOCKS * MLP_MAXSP * MLP_STRIDE + MLP_MAXSP * MLP_STRIDE + 2 * MLP_BLOCKS +
    256 * (MLP_MAXSP * (MLP_NF * 3 + 1));
static __device__ __align__(256) float scratch[MLP_SCRATCH_FLOATS];

constexpr int MLP_MAX_DEVICES = 64;
std::mutex scratch_mutex;
float* scratch_ptr[MLP_MAX_DEVICES] = {};

// Device address of this device's scratch array, looked up once per device
// (with that device current) on the first call.
int scratch_address(float** out) {
    int dev = 0;
    QEQ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MLP_MAX_DEVICES) return QEQ_EINVAL;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        QEQ_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        scratch_ptr[dev] = static_cast<float*>(p);
    }
    *out = scratch_ptr[dev];
    return QEQ_OK;
}

int train_step_impl(const float* G, const int32_t* species, const double* target, int32_t n, int32_t n_species,
                    const float* stats, float* params, float* adam_m, float* adam_v, int32_t step, float lr,
                    float* workspace, float* loss, float* grad_out, hipStream_t s) {
    const int np = n_species * MLP_STRIDE;
    float* gpart = workspace;
    float* grad = workspace + (size_t)MLP_BLOCKS * np;
    double* lpart = reinterpret_cast<double*>(grad + np + (np & 1));
    hipLaunchKernelGGL(k_mlp<true>, dim3(MLP_BLOCKS), dim3(256), 0, s, G, species, target, n, n_species, params,
                       stats, nullptr, gpart, lpart, 1.f / (float)n);
    hipLaunchKernelGGL(k_grad_reduce, dim3((np + 255) / 256), dim3(256), 0, s, gpart, MLP_BLOCKS, np, grad,
                       lpart, loss);
    if (grad_out) QEQ_HIP(hipMemcpyAsync(grad_out, grad, sizeof(float) * np, hipMemcpyDeviceToDevice, s));
    if (step > 0)
        hipLaunchKernelGGL(k_adam, dim3((np + 255) / 256), dim3(256), 0, s, params, grad, adam_m, adam_v, np, step,
                           lr);
    return qeq_check(hipGetLastError());
}

}  // namespace

int launch_descriptors(qeq_plan* pl, const double* weights, int nf, const double* centers, double width, double rc,
                       float* G) {
    if (nf < 1 || nf > 32 || !(width > 0.0) || !(rc > 0.0) || rc > pl->kp.rc) return QEQ_EINVAL;
    DescParams d;
    d.nf = nf;
    for (int m = 0; m < 32; ++m) d.centers[m] = m < nf ? (float)centers[m] : 0.f;
    d.eta = (float)(1.0 / (2.0 * width * width));
    d.rc = (float)rc;
    const int nb = (int)(((size_t)pl->kp.n * DESC_G + QEQ_BLOCK - 1) / QEQ_BLOCK);
    hipLaunchKernelGGL(k_descriptors, dim3(nb), dim3(QEQ_BLOCK), 0, pl->stream, pl->kp.n, d,
                       pl->rowptr, pl->col, pl->pdr, pl->perm, weights, G);
    return qeq_check(hipGetLastError());
}

extern "C" {

int64_t mlp_workspace_floats(int32_t n_species) {
    if (n_species < 1 || n_species > MLP_MAXSP) return -1;
    const int64_t np = (int64_t)n_species * MLP_STRIDE;
    return (int64_t)MLP_BLOCKS * np + np + 2 * MLP_BLOCKS + 256 * (MLP_MAXSP * (MLP_NF * 3 + 1));
}

int mlp_feature_stats(const float* G, const int32_t* species, int32_t n, int32_t n_species, float* stats,
                      float* workspace, void* stream) {
    if (!G || !species || !stats || !workspace || n < 1 || n_species < 1 || n_species > MLP_MAXSP)
        return QEQ_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int nblk = 256;
    hipLaunchKernelGGL(k_feat_partial, dim3(nblk), dim3(256), 0, s, G, species, n, n_species, workspace);
    hipLaunchKernelGGL(k_feat_finish, dim3(1), dim3(MLP_MAXSP * MLP_NF), 0, s, workspace, nblk, n_species,
                       stats);
    return qeq_check(hipGetLastError());
}

int mlp_forward(const float* G, const int32_t* species, int32_t n, int32_t n_species, const float* params,
                const float* stats, double* out, void* stream) {
    if (!G || !species || !params || !stats || !out || n < 1 || n_species < 1 || n_species > MLP_MAXSP)
        return QEQ_EINVAL;
    const int ntiles = (n + 15) / 16;
    int nblk = (ntiles + 3) / 4;
    if (nblk > 2048) nblk = 2048;
    hipLaunchKernelGGL(k_mlp<false>, dim3(nblk), dim3(256), 0, (hipStream_t)stream, G, species, nullptr, n,
                       n_species, params, stats, out, nullptr, nullptr, 0.f);
    return qeq_check(hipGetLastError());
}

int mlp_train_step(const float* G, const int32_t* species, const double* target, int32_t n, int32_t n_species,
                   const float* stats, float* params, float* adam_m, float* adam_v, int32_t step, float lr,
                   float* workspace, int64_t workspace_floats, float* loss, float* grad_out, void* stream) {
    if (!G || !species || !target || !stats || !params || !adam_m || !adam_v || !workspace || n < 1 ||
        n_species < 1 || n_species > MLP_MAXSP || step < 0)
        return QEQ_EINVAL;
    if (workspace_floats < mlp_workspace_floats(n_species)) return QEQ_EINVAL;
    return train_step_impl(G, species, target, n, n_species, stats, params, adam_m, adam_v, step, lr, workspace,
                           loss, grad_out, (hipStream_t)stream);
}

int mlp_train_step_noalloc(const float* G, const int32_t* species, const double* target, int32_t n,
                           int32_t n_species, const float* stats, float* params, float* adam_m, float* adam_v,
                           int32_t step, float lr, float* loss, float* grad_out, void* stream) {
    if (!G || !species || !target || !stats || !params || !adam_m || !adam_v || n < 1 || n_species < 1 ||
        n_species > MLP_MAXSP || step < 0)
        return QEQ_EINVAL;
    if (mlp_workspace_floats(n_species) > MLP_SCRATCH_FLOATS) return QEQ_EINVAL;
    float* ws = nullptr;
    QEQ_TRY(scratch_address(&ws));
    return train_step_impl(G, species, target, n, n_species, stats, params, adam_m, adam_v, step, lr, ws, loss,
                           grad_out, (hipStream_t)stream);
}

}  // extern "C"
