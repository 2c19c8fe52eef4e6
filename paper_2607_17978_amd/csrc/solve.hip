// Back-interpolation, real-space sparse product, projected Jacobi-preconditioned
// CG (FP64 vectors and reductions) and the final energies / forces.
//
// CG works on the constraint plane sum(q) = Q_tot (paper, eq. 4G_qeq_prime):
// the residual r = -(A q + chi_eff) is kept with zero mean, the preconditioned
// residual z = D^-1 r - c D^-1 1 with c = sum(D^-1 r) / sum(D^-1) has zero sum,
// so every search direction stays on the plane.  Per iteration:
//   mesh (5 passes) -> k_interp (y = A p, partial p.y and sum y)
//   -> k_cg_update (alpha, q, r, partial sums for z) -> k_cg_dir (beta, p).
// The background term of charged cells is a rank-two update whose effect on
// the constrained solution is the shift chi_eff = chi + (2 pi / V) Q sigma^2.
#include <math.h>

#include "internal.h"

namespace {

// y_i = sum_g theta_i(g) phi(g) + sum_j K_ij v_j + d_i v_i (+ J_i v_i)
// and, in FINAL mode, the force on atom i.  One wave per atom: lane
// (k2, k3) < p^2 gathers the p grid values along axis 1 at that (k2, k3)
// (adjacent lanes read adjacent addresses), all 64 lanes then stride over the
// atom's pair-list row; the partial sums are reduced across the wave.  (One
// thread per atom would leave the chip with a few hundred waves and 216
// dependent gathers each.)
template <int MODE, int PC>
__global__ __launch_bounds__(QEQ_BLOCK) void k_interp(
    KParams k, const double* __restrict__ src, const double* __restrict__ yrec, double* __restrict__ dst,
    const float* __restrict__ grid,
    const int* __restrict__ home, const float* __restrict__ wts, const float* __restrict__ dwts,
    const int* __restrict__ rowptr, const int* __restrict__ col, const float* __restrict__ kval,
    const float4* __restrict__ pdr, const double* __restrict__ dself, const double* __restrict__ Jv,
    const double* __restrict__ chi_raw, const double* __restrict__ chi_eff, const double* __restrict__ sig,
    const double* __restrict__ selfgrad, double* __restrict__ forces, double* __restrict__ gvec,
    double* __restrict__ part, CgScalars* __restrict__ sc, int parity, const float* __restrict__ mpart) {
    if (MODE == QEQ_MODE_CG && sc->done) return;
    constexpr bool FIN = MODE == QEQ_MODE_FINAL;
    const int lane = threadIdx.x & 63;
    const int p = PC ? PC : k.p;
    const int nwaves = gridDim.x * (blockDim.x >> 6);
    double acc[QEQ_NPART];
#pragma unroll
    for (int t = 0; t < QEQ_NPART; ++t) acc[t] = 0.0;
    // waves stride over atoms; the loop trip count is uniform across the block
    const int rounds = (k.n + nwaves - 1) / nwaves;
    const int wave = (xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) >> 6;
    // the row bounds and home indices of the next round's atom are loaded
    // one round ahead, so that each round starts with its first load level
    // already in flight
    int nx_e0 = 0, nx_e1 = 0, nx_h1 = 0, nx_h2 = 0, nx_h3 = 0;
    if (wave < k.n) {
        nx_e0 = rowptr[wave];
        nx_e1 = rowptr[wave + 1];
        nx_h1 = home[4 * wave];
        nx_h2 = home[4 * wave + 1];
        nx_h3 = home[4 * wave + 2];
    }
    for (int rnd = 0; rnd < rounds; ++rnd) {
    const int i = rnd * nwaves + wave;
    // per-lane partials: y, du[3] (reciprocal gradient / q), fr[3] (pair gradient / q)
    double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const bool active = i < k.n;
    const int cur_e0 = nx_e0, cur_e1 = nx_e1, cur_h1 = nx_h1, cur_h2 = nx_h2, cur_h3 = nx_h3;
    if (active) {
        // Loads are issued in three dependent levels so that their latencies
        // overlap (the memory counter retires loads in issue order): the row
        // bounds and home indices; then the first 64 pairs' columns and
        // kernel values, the lane's grid line and weights; then the source
        // values of those columns.  Arithmetic follows.
        constexpr int PM = PC ? PC : QEQ_MAXP;
        // mesh part already interpolated by the fused complex-to-real pass:
        // lanes < 2p hold its per-atom partials
        const bool do_recip = (k.parts & QEQ_PART_RECIP) && lane < p * p && !mpart;
        const bool do_real = (k.parts & QEQ_PART_REAL) != 0;
        const int e0 = cur_e0, e1 = cur_e1;
        const int h1 = cur_h1, h2 = cur_h2, h3 = cur_h3;
        const int ef = e0 + lane;
        const bool has_pair = do_real && ef < e1;
        int cj = 0;
        float kv = 0.f;
        float4 d = make_float4(0.f, 0.f, 0.f, 0.f);
        if (has_pair) {
            cj = col[ef];
            kv = kval[ef];
            if (FIN) d = pdr[ef];
        }
        // lane (k2, k3), k3 fastest: the lanes of one k2 read p consecutive
        // grid values, so each load instruction touches p short runs instead
        // of p^2 scattered rows; k1 runs along the lane's line
        const int k2 = lane / p, k3 = lane - (lane / p) * p;
        const float* w = wts + (size_t)i * 3 * QEQ_MAXP;
        const float* dw = dwts + (size_t)i * 3 * QEQ_MAXP;
        float gv[PM], wk[PM], dwk[PM];
        float w2 = 0.f, w3 = 0.f, dw2 = 0.f, dw3 = 0.f;
        if (do_recip) {
            int g2 = h2 - k2;
            if (g2 < 0) g2 += k.K2;
            int g3 = h3 - k3;
            if (g3 < 0) g3 += k.K3;
            const size_t plane = (size_t)k.K2 * k.K3;
            const float* colp = grid + (size_t)g2 * k.K3 + g3;
#pragma unroll
            for (int k1 = 0; k1 < PM; ++k1) {
                if (!PC && k1 >= p) break;
                int g1 = h1 - k1;
                if (g1 < 0) g1 += k.K1;
                gv[k1] = colp[(size_t)g1 * plane];
                wk[k1] = w[k1];
                if (FIN) dwk[k1] = dw[k1];
            }
            w2 = w[QEQ_MAXP + k2];
            w3 = w[2 * QEQ_MAXP + k3];
            if (FIN) {
                dw2 = dw[QEQ_MAXP + k2];
                dw3 = dw[2 * QEQ_MAXP + k3];
            }
        }
        // next round's first load level, behind this round's second
        const int in = i + nwaves;
        if (in < k.n) {
            nx_e0 = rowptr[in];
            nx_e1 = rowptr[in + 1];
            nx_h1 = home[4 * in];
            nx_h2 = home[4 * in + 1];
            nx_h3 = home[4 * in + 2];
        }
        const double vj = has_pair ? src[cj] : 0.0;
        if (mpart && (k.parts & QEQ_PART_RECIP) && lane < 2 * p) v[0] = (double)mpart[(size_t)lane * k.n + i];
        if (do_recip) {
            float s = 0.f, s1 = 0.f;
#pragma unroll
            for (int k1 = 0; k1 < PM; ++k1) {
                if (!PC && k1 >= p) break;
                s += wk[k1] * gv[k1];
                if (FIN) s1 += dwk[k1] * gv[k1];
            }
            v[0] = (double)(w2 * w3) * (double)s;
            if (FIN) {
                v[1] = (double)(w2 * w3) * (double)s1;
                v[2] = (double)(dw2 * w3) * (double)s;
                v[3] = (double)(w2 * dw3) * (double)s;
            }
        }
        if (has_pair) {
            v[0] += (double)kv * vj;
            if (FIN) {
                const double c = (double)d.w * vj;
                v[4] += c * d.x;
                v[5] += c * d.y;
                v[6] += c * d.z;
            }
        }
        // rows of more than 64 pairs
        if (do_real) {
            for (int e = ef + 64; e < e1; e += 64) {
                const double vje = src[col[e]];
                v[0] += (double)kval[e] * vje;
                if (FIN) {
                    const float4 de = pdr[e];
                    const double c = (double)de.w * vje;
                    v[4] += c * de.x;
                    v[5] += c * de.y;
                    v[6] += c * de.z;
                }
            }
        }
    }
    v[0] = wave_sum(v[0]);
    if (FIN) {
#pragma unroll
        for (int t = 1; t < 7; ++t) v[t] = wave_sum(v[t]);
    }
    if (active && lane == 0) {
        const double vi = src[i];
        double y = v[0];
        if (yrec) y += yrec[i];   // reciprocal part computed elsewhere (direct Ewald sums)
        if (k.parts & QEQ_PART_SELF) y += dself[i] * vi;
        if (MODE == QEQ_MODE_CG) {
            y += Jv[i] * vi;
            acc[0] += vi * y;
            acc[1] += y;
        }
        dst[i] = y;
        if (FIN) {
            // forces: -dE/dr_i, with u_a = K_a s_a and s = r H^-1
            double du[3] = {v[1], v[2], v[3]};
            if (k.self_corr && (k.parts & QEQ_PART_SELF)) {
                // +1/2 q_i^2 d(theta^T Theta theta)/du cancels the mesh self-force
                for (int a = 0; a < 3; ++a) du[a] -= 0.5 * vi * selfgrad[3 * i + a];
            }
            const double Kd[3] = {(double)k.K1, (double)k.K2, (double)k.K3};
            for (int c = 0; c < 3; ++c) {
                double g = 0.0;
                for (int a = 0; a < 3; ++a) g += Kd[a] * k.Hinv[c * 3 + a] * du[a];
                forces[3 * i + c] = -vi * g - vi * v[4 + c];
            }
            const double J = Jv[i];
            const double gi = y + J * vi + chi_eff[i];
            gvec[i] = gi;
            acc[0] += vi * y;               // q.E q (no background)
            acc[1] += chi_raw[i] * vi;      // chi.q
            acc[2] += J * vi * vi;          // J q^2
            acc[3] += sig[i] * sig[i] * vi; // sigma^2 q
            acc[4] += gi;                   // sum of the gradient
        }
    }
    }   // rounds
    if (MODE != QEQ_MODE_MATVEC) {
        block_sum<5>(acc);
        if (threadIdx.x == 0) {
            for (int t = 0; t < 5; ++t) part[blockIdx.x * QEQ_NPART + t] = acc[t];
        }
    }
    (void)parity;
}

// The CG product when the mesh part arrives as interpolation partials (the
// fused complex-to-real pass): y_i = sum of the atom's 2p partials +
// sum_j K_ij v_j + d_i v_i (+ J_i v_i).  Sixteen lanes per atom (four atoms
// per wave); each lane takes every sixteenth pair of the row, with the loads
// of four pairs issued before their sums so that the column, kernel-value and
// source gathers of a row overlap; the sixteen partial sums are combined in a
// fixed butterfly order.  Same partial-sum layout as k_interp (the next CG
// kernel reduces them): 16 atoms per block and round.
template <int MODE>
__global__ __launch_bounds__(QEQ_BLOCK) void k_pairs_fused(
    KParams k, const double* __restrict__ src, double* __restrict__ dst, const int* __restrict__ rowptr,
    const int* __restrict__ col, const float* __restrict__ kval, const double* __restrict__ dself,
    const double* __restrict__ Jv, const float* __restrict__ mpart, double* __restrict__ part,
    CgScalars* __restrict__ sc) {
    const int done = MODE == QEQ_MODE_CG ? sc->done : 0;
    constexpr int G = 16;
    const int lane = threadIdx.x & (G - 1);
    const int grp = (xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) / G;
    const int ngrp = gridDim.x * (blockDim.x / G);
    const int n = k.n;
    const bool do_real = (k.parts & QEQ_PART_REAL) != 0;
    const bool do_recip = (k.parts & QEQ_PART_RECIP) != 0 && lane < 2 * k.p;
    const bool do_self = (k.parts & QEQ_PART_SELF) != 0;
    // The loads of a round that do not depend on its row (the row bounds, the
    // mesh partial, the atom's own terms) are issued one round ahead; the
    // first round's before the converged flag is tested, so that they share
    // its memory round trip.
    int e0n = 0, e1n = 0;
    float mpn = 0.f;
    double vin = 0.0, dsn = 0.0, jvn = 0.0;
    auto fetch = [&](int i) {
        if (i < n) {
            e0n = rowptr[i];
            e1n = rowptr[i + 1];
            mpn = do_recip ? mpart[(size_t)lane * n + i] : 0.f;
            if (lane == 0) {
                vin = src[i];
                if (do_self) dsn = dself[i];
                if (MODE == QEQ_MODE_CG) jvn = Jv[i];
            }
        }
    };
    fetch(grp);
    if (done) return;
    double acc[2] = {0.0, 0.0};
    const int rounds = (n + ngrp - 1) / ngrp;
    for (int rnd = 0; rnd < rounds; ++rnd) {
        const int i = rnd * ngrp + grp;
        const int e0 = e0n, e1 = e1n;
        const float mp = mpn;
        const double vi = vin, ds = dsn, jv = jvn;
        fetch(i + ngrp);
        double v = 0.0;
        if (i < n) {
            if (do_real) {
                for (int base = e0 + lane; base < e1; base += 4 * G) {
                    int cj[4];
                    float kv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int e = base + u * G;
                        cj[u] = e < e1 ? col[e] : -1;
                        kv[u] = e < e1 ? kval[e] : 0.f;
                    }
                    double vj[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) vj[u] = cj[u] >= 0 ? src[cj[u]] : 0.0;
#pragma unroll
                    for (int u = 0; u < 4; ++u) v += (double)kv[u] * vj[u];
                }
            }
            v += (double)mp;
        }
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
        if (i < n && lane == 0) {
            double y = v;
            if (do_self) y += ds * vi;
            if (MODE == QEQ_MODE_CG) {
                y += jv * vi;
                acc[0] += vi * y;
                acc[1] += y;
            }
            dst[i] = y;
        }
    }
    if (MODE == QEQ_MODE_CG) {
        block_sum<2>(acc);
        if (threadIdx.x == 0) {
            part[blockIdx.x * QEQ_NPART] = acc[0];
            part[blockIdx.x * QEQ_NPART + 1] = acc[1];
            for (int t = 2; t < 5; ++t) part[blockIdx.x * QEQ_NPART + t] = 0.0;
        }
    }
}

// q <- q0 (original order, gathered to sorted) or Q/N; partial sum(q).
__global__ void k_cg_init_q(KParams k, const double* __restrict__ q0, const int* __restrict__ perm,
                            double* __restrict__ q, double* __restrict__ part, CgScalars* sc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double v[1] = {0.0};
    if (i < k.n) {
        double x = q0 ? q0[perm[i]] : k.q_tot / (double)k.n;
        if (!isfinite(x)) {
            x = k.q_tot / (double)k.n;
            atomicOr(&sc->err, QEQ_ERRBIT_INPUT);
        }
        q[i] = x;
        v[0] = x;
    }
    block_sum<1>(v);
    if (threadIdx.x == 0) part[blockIdx.x * QEQ_NPART] = v[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->done = 0;
        sc->iters = 0;
    }
}

template <int NV>
__device__ __forceinline__ void reduce_strided(const double* part, int nparts, double* out) {
    __shared__ double tot[NV];
    double v[NV];
#pragma unroll
    for (int t = 0; t < NV; ++t) v[t] = 0.0;
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
#pragma unroll
        for (int t = 0; t < NV; ++t) v[t] += part[b * QEQ_NPART + t];
    }
    block_sum<NV>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int t = 0; t < NV; ++t) tot[t] = v[t];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NV; ++t) out[t] = tot[t];
    __syncthreads();
}

// shift q onto the constraint plane sum(q) = Q_tot
__global__ void k_cg_project_q(KParams k, double* __restrict__ q, const double* __restrict__ part,
                               int nparts) {
    double tot[1];
    reduce_strided<1>(part, nparts, tot);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k.n) q[i] += (k.q_tot - tot[0]) / (double)k.n;
}

// r = -(chi_eff + A q) with zero mean (y = A q and its partial sums from the
// preceding matvec); partial sums of D^-1 r, r^2 / D and r^2.
__global__ void k_cg_init_r(KParams k, const double* __restrict__ y, const double* __restrict__ chi,
                            const double* __restrict__ dinv, const double* __restrict__ q,
                            double* __restrict__ r, const double* __restrict__ part_in, int nparts,
                            double* __restrict__ part_out, const CgScalars* __restrict__ sc) {
    double tot[2];
    reduce_strided<2>(part_in, nparts, tot);
    const double shift = (sc->chi_sum + tot[1]) / (double)k.n;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < k.n) {
        const double ri = -chi[i] - y[i] + shift;
        r[i] = ri;
        const double di = dinv[i];
        acc[0] = di * ri;
        acc[1] = di * ri * ri;
        acc[2] = ri * ri;
        acc[3] = chi[i] * q[i];   // for the energy of the starting point
    }
    block_sum<4>(acc);
    if (threadIdx.x == 0) {
        for (int t = 0; t < 4; ++t) part_out[blockIdx.x * QEQ_NPART + t] = acc[t];
    }
}

// Energy of the starting point on the constraint plane, 1/2 q.(A q) + chi_eff.q
// (up to a constant that is the same for every feasible q), from the partial
// sums of the initial matvec (slot 0: q.A q) and of k_cg_init_r (slot 3).
__global__ void k_start_energy(const double* __restrict__ part_mv, int n_mv, const double* __restrict__ part_r,
                               int n_r, CgScalars* sc) {
    double a[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < n_mv; b += blockDim.x) a[0] += part_mv[b * QEQ_NPART];
    for (int b = threadIdx.x; b < n_r; b += blockDim.x) a[1] += part_r[b * QEQ_NPART + 3];
    block_sum<2>(a);
    if (threadIdx.x == 0) sc->e_start = 0.5 * a[0] + a[1];
}

// Loads of NV per-block partial sums (layout part[b * QEQ_NPART + t]) into
// this thread's running sums, in the order reduce_strided adds them; the
// block sum follows in block_total.
template <int NV>
__device__ __forceinline__ void load_strided(const double* part, int nparts, double* v) {
#pragma unroll
    for (int t = 0; t < NV; ++t) v[t] = 0.0;
#pragma unroll 4
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
#pragma unroll
        for (int t = 0; t < NV; ++t) v[t] += part[b * QEQ_NPART + t];
    }
}

template <int NV>
__device__ __forceinline__ void block_total(double* v) {
    __shared__ double tot[NV];
    block_sum<NV>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int t = 0; t < NV; ++t) tot[t] = v[t];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NV; ++t) v[t] = tot[t];
}

// alpha = r.z / p.A p; q += alpha p; r -= alpha (A p - mean(A p)).
// Every load is issued before the converged flag is tested (the flag is the
// same for all blocks), so that the flag, the partial sums and the vector
// elements arrive in one memory round trip rather than three.
// With the spectral preconditioner (sd != nullptr) it also writes that
// preconditioner's input u = D'^-1/2 r (as k_spc_u does; the padding past n
// keeps the zeros of the solve's first application).
__global__ void k_cg_update(KParams k, const double* __restrict__ p, const double* __restrict__ y,
                            const double* __restrict__ dinv, double* __restrict__ q, double* __restrict__ r,
                            const double* __restrict__ part_in, int nparts, double* __restrict__ part_out,
                            CgScalars* sc, int parity, const float* __restrict__ sd, float* __restrict__ u) {
    const int done = sc->done;
    const double rzp = sc->rz[parity];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double pi = 0.0, yi = 0.0, qi = 0.0, ri = 0.0, di = 0.0;
    if (i < k.n) {
        pi = p[i];
        yi = y[i];
        qi = q[i];
        ri = r[i];
        di = dinv[i];
    }
    double tot[2];
    load_strided<2>(part_in, nparts, tot);
    if (done) return;
    block_total<2>(tot);
    const double alpha = rzp / tot[0];
    const double ymean = tot[1] / (double)k.n;
    double acc[3] = {0.0, 0.0, 0.0};
    if (i < k.n) {
        q[i] = qi + alpha * pi;
        ri -= alpha * (yi - ymean);
        r[i] = ri;
        if (u) u[i] = (float)((double)sd[i] * ri);
        acc[0] = di * ri;
        acc[1] = di * ri * ri;
        acc[2] = ri * ri;
    }
    block_sum<3>(acc);
    if (threadIdx.x == 0) {
        for (int t = 0; t < 3; ++t) part_out[blockIdx.x * QEQ_NPART + t] = acc[t];
        if (blockIdx.x == 0) {
            sc->alpha = alpha;
            sc->iters += 1;
        }
    }
}

// c = sum(D^-1 r) / sum(D^-1) projects the preconditioned residual onto sum = 0,
// r.z = sum(r^2/D) - c sum(D^-1 r), beta = r.z / r.z_old, p = D^-1 (r - c) + beta p;
// the relative residual ||r|| / ||P chi_eff|| decides convergence.  Loads
// are issued before the converged flag is tested, as in k_cg_update.
__global__ void k_cg_dir(KParams k, const double* __restrict__ r, const double* __restrict__ dinv,
                         double* __restrict__ p, const double* __restrict__ part_in, int nparts,
                         CgScalars* sc, int parity, int init) {
    const int done = sc->done;
    const double rz_old = sc->rz[parity], dinv_sum = sc->dinv_sum, chi_norm = sc->chi_norm;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double ri = 0.0, di = 0.0, pi = 0.0;
    if (i < k.n) {
        ri = r[i];
        di = dinv[i];
        pi = p[i];
    }
    double tot[3];
    load_strided<3>(part_in, nparts, tot);
    if (done) return;
    block_total<3>(tot);
    const double c = tot[0] / dinv_sum;
    const double rz = tot[1] - c * tot[0];
    const double beta = init ? 0.0 : rz / rz_old;
    const double res = chi_norm > 0.0 ? sqrt(tot[2]) / chi_norm : sqrt(tot[2]);
    // the first direction does not use p: its memory may hold anything (0 * NaN = NaN)
    if (i < k.n) p[i] = di * (ri - c) + (init ? 0.0 : beta * pi);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->rz[parity ^ 1] = rz;
        sc->res = res;
        if (res <= k.tol || !(res == res)) sc->done = 1;
    }
}

// Final: reduce energy partials, the mean gradient (= mu up to the background
// constant) and the deviation of the gradient from it; scatter outputs.
__global__ void k_final2(KParams k, const double* __restrict__ q_s, const double* __restrict__ f_s,
                         const double* __restrict__ gvec, const int* __restrict__ perm,
                         double* __restrict__ q_out, double* __restrict__ f_out,
                         const double* __restrict__ part_in, int nparts, double* __restrict__ part_out) {
    double tot[5];
    reduce_strided<5>(part_in, nparts, tot);
    const double gmean = tot[4] / (double)k.n;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double acc[1] = {0.0};
    if (i < k.n) {
        int o = perm[i];
        if (q_out) q_out[o] = q_s[i];
        if (f_out) {
            f_out[3 * o] = f_s[3 * i];
            f_out[3 * o + 1] = f_s[3 * i + 1];
            f_out[3 * o + 2] = f_s[3 * i + 2];
        }
        double d = gvec[i] - gmean;
        acc[0] = d * d;
    }
    block_sum<1>(acc);
    if (threadIdx.x == 0) part_out[blockIdx.x * QEQ_NPART] = acc[0];
}

__global__ void k_final3(KParams k, const double* __restrict__ part5, int nparts5,
                         const double* __restrict__ part1, int nparts1, const CgScalars* __restrict__ sc,
                         double* __restrict__ out, double* __restrict__ energies) {
    double tot[5];
    reduce_strided<5>(part5, nparts5, tot);
    double dev[1];
    reduce_strided<1>(part1, nparts1, dev);
    if (threadIdx.x == 0) {
        const double Q = k.q_tot;
        const double S2 = tot[3];
        const double e_bg = -0.5 * k.bg_pref * (k.eta * k.eta * Q * Q - 2.0 * Q * S2);
        const double e_elec = 0.5 * tot[0] + e_bg;
        const double e_qeq = e_elec + tot[1] + 0.5 * tot[2];
        const double mu = tot[4] / (double)k.n - k.bg_pref * (k.eta * k.eta * Q - S2);
        const double tres = sc->chi_norm > 0.0 ? sqrt(dev[0]) / sc->chi_norm : sqrt(dev[0]);
        out[0] = e_qeq;
        out[1] = e_elec;
        out[2] = mu;
        out[3] = tres;
        if (energies) {
            energies[0] = e_qeq;
            energies[1] = e_elec;
        }
    }
}

// Matrix-vector entry point: permute the input to sorted order, add the
// background term, permute the output back.
__global__ void k_perm_in(int n, const double* __restrict__ v, const int* __restrict__ perm,
                          const double* __restrict__ sig, double* __restrict__ vs, double* __restrict__ part) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double acc[2] = {0.0, 0.0};
    if (i < n) {
        double x = v[perm[i]];
        vs[i] = x;
        acc[0] = x;
        acc[1] = sig[i] * sig[i] * x;
    }
    block_sum<2>(acc);
    if (threadIdx.x == 0) {
        part[blockIdx.x * QEQ_NPART] = acc[0];
        part[blockIdx.x * QEQ_NPART + 1] = acc[1];
    }
}

__global__ void k_perm_out(KParams k, const double* __restrict__ ys, const int* __restrict__ perm,
                           const double* __restrict__ sig, double* __restrict__ y,
                           const double* __restrict__ part, int nparts) {
    double tot[2];
    reduce_strided<2>(part, nparts, tot);
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k.n) return;
    double v = ys[i];
    if (k.parts & QEQ_PART_BG) {
        double s2 = sig[i] * sig[i];
        v -= k.bg_pref * ((k.eta * k.eta - s2) * tot[0] - tot[1]);
    }
    y[perm[i]] = v;
}

}  // namespace

static double* part_buf(qeq_plan* pl, int which) { return pl->part + (size_t)which * pl->nblk_max * QEQ_NPART; }

template <int MODE>
static void interp_launch(qeq_plan* pl, const double* src, double* dst, double* part, int parity,
                          hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, const float* mpart = nullptr) {
    const int nb = interp_blocks(pl->kp.n);   // one wave per atom
#define QEQ_INTERP_ARGS                                                                              \
    dim3(nb), dim3(QEQ_BLOCK), 0, pl->stream, ev0, ev1, 0, pl->kp, src,                                  \
        (pl->ew_active ? (const double*)pl->ew_yrec : pl->pw_active ? (const double*)pl->pw_y : nullptr), dst, pl->grid_r, pl->home, pl->wts, \
        pl->dwts, pl->rowptr, pl->col, pl->kval, pl->pdr, pl->dself, pl->Jv, pl->chi_raw, pl->chi,   \
        pl->sig, pl->selfgrad, pl->fdst, pl->gtmp, part, pl->sc, parity, mpart
    if (pl->kp.p == 6)
        hipExtLaunchKernelGGL((k_interp<MODE, 6>), QEQ_INTERP_ARGS);
    else
        hipExtLaunchKernelGGL((k_interp<MODE, 0>), QEQ_INTERP_ARGS);
#undef QEQ_INTERP_ARGS
}

int launch_interp(qeq_plan* pl, const double* src, double* dst, int mode, int parity, const float* mpart) {
    double* part = part_buf(pl, 0);
    ProfScope ps(pl, mode == QEQ_MODE_CG ? PK_INTERP : PK_COUNT);
    if (mpart && (mode == QEQ_MODE_CG || mode == QEQ_MODE_MATVEC) && !pl->ew_active && !pl->pw_active) {
        const int nb = interp_blocks(pl->kp.n);   // the partial-sum count the CG kernels expect
        if (mode == QEQ_MODE_CG)
            hipExtLaunchKernelGGL(k_pairs_fused<QEQ_MODE_CG>, dim3(nb), dim3(QEQ_BLOCK), 0, pl->stream, ps.start(),
                                  ps.stop(), 0, pl->kp, src, dst, pl->rowptr, pl->col, pl->kval, pl->dself,
                                  pl->Jv, mpart, part, pl->sc);
        else
            hipExtLaunchKernelGGL(k_pairs_fused<QEQ_MODE_MATVEC>, dim3(nb), dim3(QEQ_BLOCK), 0, pl->stream,
                                  nullptr, nullptr, 0, pl->kp, src, dst, pl->rowptr, pl->col, pl->kval, pl->dself,
                                  pl->Jv, mpart, part, pl->sc);
        return qeq_check(hipGetLastError());
    }
    if (mode == QEQ_MODE_CG)
        interp_launch<QEQ_MODE_CG>(pl, src, dst, part, parity, ps.start(), ps.stop(), mpart);
    else if (mode == QEQ_MODE_MATVEC)
        interp_launch<QEQ_MODE_MATVEC>(pl, src, dst, part, parity, nullptr, nullptr, mpart);
    else if (!mpart)
        interp_launch<QEQ_MODE_FINAL>(pl, src, dst, part, parity);
    else
        return QEQ_EINVAL;   // forces need the potential grid
    return qeq_check(hipGetLastError());
}

int launch_cg_init_q(qeq_plan* pl, const double* q0) {
    const int nb = nblocks(pl->kp.n);
    hipLaunchKernelGGL(k_cg_init_q, dim3(nb), dim3(QEQ_BLOCK), 0, pl->stream, pl->kp, q0, pl->perm,
                       pl->q, part_buf(pl, 1), pl->sc);
    hipLaunchKernelGGL(k_cg_project_q, dim3(nb), dim3(QEQ_BLOCK), 0, pl->stream, pl->kp, pl->q,
                       part_buf(pl, 1), nb);
    return qeq_check(hipGetLastError());
}

// Block width of the CG vector kernels.  Each block reduces all of the
// product's partial sums (4,096 of them at 131,072 atoms), so large systems
// take fewer, wider blocks (131,072 atoms: 26.58 -> 26.46 ms per solve; at
// 32,768 atoms the wide blocks were slower, 5.26 -> 5.44 ms).
static int vblock(int n) { return n >= 65536 ? 1024 : QEQ_VBLOCK; }

int launch_cg_init_r(qeq_plan* pl) {
    const int vb = vblock(pl->kp.n), nb = nblocks(pl->kp.n, vb);
    hipLaunchKernelGGL(k_cg_init_r, dim3(nb), dim3(vb), 0, pl->stream, pl->kp, pl->y, pl->chi,
                       pl->dinv, pl->q, pl->r, part_buf(pl, 0), interp_blocks(pl->kp.n), part_buf(pl, 1), pl->sc);
    return qeq_check(hipGetLastError());
}

int launch_start_energy(qeq_plan* pl) {
    hipLaunchKernelGGL(k_start_energy, dim3(1), dim3(QEQ_BLOCK), 0, pl->stream, part_buf(pl, 0),
                       interp_blocks(pl->kp.n), part_buf(pl, 1), nblocks(pl->kp.n, vblock(pl->kp.n)), pl->sc);
    return qeq_check(hipGetLastError());
}

int launch_cg_update(qeq_plan* pl, int parity) {
    const int vb = vblock(pl->kp.n), nb = nblocks(pl->kp.n, vb);
    ProfScope ps(pl, PK_CG_UPDATE);
    hipExtLaunchKernelGGL(k_cg_update, dim3(nb), dim3(vb), 0, pl->stream, ps.start(), ps.stop(), 0, pl->kp,
                       pl->pvec, pl->y,
                       pl->dinv, pl->q, pl->r, part_buf(pl, 0), interp_blocks(pl->kp.n), part_buf(pl, 1),
                       pl->sc, parity, pl->spc_active ? pl->spc_sd : nullptr,
                       pl->spc_active ? pl->spc_u : nullptr);
    return qeq_check(hipGetLastError());
}

int launch_cg_dir(qeq_plan* pl, int parity, int init) {
    const int vb = vblock(pl->kp.n), nb = nblocks(pl->kp.n, vb);
    ProfScope ps(pl, PK_CG_DIR);
    hipExtLaunchKernelGGL(k_cg_dir, dim3(nb), dim3(vb), 0, pl->stream, ps.start(), ps.stop(), 0, pl->kp,
                       pl->r, pl->dinv,
                       pl->pvec, part_buf(pl, 1), nb, pl->sc, parity, init);
    return qeq_check(hipGetLastError());
}

static void final_tail(qeq_plan* pl, double* q_out, double* energies, double* forces_out, hipEvent_t ev1) {
    const int nb = nblocks(pl->kp.n);
    double* part = part_buf(pl, 0);
    hipLaunchKernelGGL(k_final2, dim3(nb), dim3(QEQ_BLOCK), 0, pl->stream, pl->kp, pl->q, pl->fdst,
                       pl->gtmp, pl->perm, q_out, forces_out, part, interp_blocks(pl->kp.n), part_buf(pl, 1));
    hipExtLaunchKernelGGL(k_final3, dim3(1), dim3(QEQ_BLOCK), 0, pl->stream, nullptr, ev1, 0, pl->kp, part,
                          interp_blocks(pl->kp.n), part_buf(pl, 1), nb, pl->sc, pl->final_dev, energies);
}

int launch_final(qeq_plan* pl, double* q_out, double* energies, double* forces_out) {
    double* part = part_buf(pl, 0);
    ProfScope ps(pl, PK_FINAL);
    interp_launch<QEQ_MODE_FINAL>(pl, pl->q, pl->y, part, 0, ps.start(), nullptr);
    if (pl->ew_active) QEQ_TRY(launch_ew_forces_add(pl));   // reciprocal forces of the direct sums
    if (pl->pw_active) QEQ_TRY(launch_pw_forces_add(pl));   // forces of the Gaussian-on-grid operator
    final_tail(pl, q_out, energies, forces_out, ps.stop());
    return qeq_check(hipGetLastError());
}

// Energies, mu, true residual and the scatter to caller order from partial
// sums of a final product that another operator (the direct pair sum) wrote
// in the same slots.
int launch_final_tail(qeq_plan* pl, double* q_out, double* energies, double* forces_out) {
    final_tail(pl, q_out, energies, forces_out, nullptr);
    return qeq_check(hipGetLastError());
}

int launch_matvec_io(qeq_plan* pl, const double* v_orig, double* y_orig, int stage) {
    int nb = nblocks(pl->kp.n);
    if (stage == 0) {
        hipLaunchKernelGGL(k_perm_in, dim3(nb), dim3(QEQ_BLOCK), 0, pl->stream, pl->kp.n, v_orig, pl->perm,
                           pl->sig, pl->pvec, part_buf(pl, 1));
    } else {
        hipLaunchKernelGGL(k_perm_out, dim3(nb), dim3(QEQ_BLOCK), 0, pl->stream, pl->kp, pl->y, pl->perm,
                           pl->sig, y_orig, part_buf(pl, 1), nb);
    }
    return qeq_check(hipGetLastError());
}
