// Adjoint backward of the QEq solve (SI "Fourth-Generation HDNNPs and Charge
// Equilibration", eq. 4g_force_trick: one extra linear system instead of 3N
// charge derivatives).  For a loss L(q, E_elec, E_QEq):
//   g = dL/dq + dL/dE_elec (E q)                       (adjoint right-hand side)
//   [A 1; 1^T 0] [a; nu] = [g; 0]                      (same operator, same CG)
//   dL/dchi = -a + dL/dE_QEq q
//   dL/dJ   = -a q + dL/dE_QEq q^2 / 2
//   dL/dr   = (dL/dE_elec + dL/dE_QEq) dE_elec/dr|_q - d(a^T E q)/dr|_{a,q}
// The bilinear derivative needs the potentials of q and of a:
//   d(a^T E_rec q)/du_i = a_i sum_g dtheta_i(g)/du phi_q(g) + q_i sum_g dtheta_i(g)/du phi_a(g)
// plus the pair term sum_j (a_i q_j + q_i a_j) K'(r_ij) r_ij / r and the
// position dependence of the mesh self-correction (-a_i q_i d(theta^T Theta theta)/du).
#include <math.h>

#include "internal.h"

namespace {

// g_i (sorted) and the adjoint "electronegativity" -g_i; partial sums laid out
// like the solve's setup (slot 0: sum of the right-hand side, slot 1: sum 1/D).
__global__ void k_adj_rhs(KParams k, const double* __restrict__ dLdq, const int* __restrict__ perm,
                          const double* __restrict__ y, const double* __restrict__ sig,
                          const double* __restrict__ dinv, double dLdEelec, double* __restrict__ chi_adj,
                          double* __restrict__ part) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double acc[2] = {0.0, 0.0};
    if (i < k.n) {
        const double s2 = sig[i] * sig[i];
        // (E q)_i up to a constant: mesh + pairs + self (y) + sigma-dependent background
        const double eq = y[i] + k.bg_pref * k.q_tot * s2;
        const double g = (dLdq ? dLdq[perm[i]] : 0.0) + dLdEelec * eq;
        chi_adj[i] = -g;
        acc[0] = -g;
        acc[1] = dinv[i];
    }
    block_sum<2>(acc);
    if (threadIdx.x == 0) {
        part[blockIdx.x * QEQ_NPART + 0] = acc[0];
        part[blockIdx.x * QEQ_NPART + 1] = acc[1];
    }
}

// Wave per atom: t_i = sum_g dtheta_i(g)/du_a phi(g), a = 1..3.
template <int PC>
__device__ __forceinline__ void recip_grad_wave(const KParams& k, int i, int lane, const float* __restrict__ grid,
                                                const int* __restrict__ home, const float* __restrict__ wts,
                                                const float* __restrict__ dwts, double* t) {
    const int p = PC ? PC : k.p;
    t[0] = t[1] = t[2] = 0.0;
    if (lane < p * p) {
        const int k1 = lane / p, k2 = lane - (lane / p) * p;
        const int h1 = home[4 * i], h2 = home[4 * i + 1], h3 = home[4 * i + 2];
        const float* w = wts + (size_t)i * 3 * QEQ_MAXP;
        const float* dw = dwts + (size_t)i * 3 * QEQ_MAXP;
        int g1 = h1 - k1;
        if (g1 < 0) g1 += k.K1;
        int g2 = h2 - k2;
        if (g2 < 0) g2 += k.K2;
        const float* row = grid + ((size_t)g1 * k.K2 + g2) * k.K3;
        float s = 0.f, s3 = 0.f;
        for (int k3 = 0; k3 < p; ++k3) {
            int g3 = h3 - k3;
            if (g3 < 0) g3 += k.K3;
            const float gv = row[g3];
            s += w[2 * QEQ_MAXP + k3] * gv;
            s3 += dw[2 * QEQ_MAXP + k3] * gv;
        }
        const float w1 = w[k1], w2 = w[QEQ_MAXP + k2];
        t[0] = (double)(dw[k1] * w2) * (double)s;
        t[1] = (double)(w1 * dw[QEQ_MAXP + k2]) * (double)s;
        t[2] = (double)(w1 * w2) * (double)s3;
    }
    t[0] = wave_sum(t[0]);
    t[1] = wave_sum(t[1]);
    t[2] = wave_sum(t[2]);
}

template <int PC>
__global__ __launch_bounds__(QEQ_BLOCK) void k_grad_recip(KParams k, const float* __restrict__ grid,
                                                         const int* __restrict__ home,
                                                         const float* __restrict__ wts,
                                                         const float* __restrict__ dwts,
                                                         double* __restrict__ tq) {
    const int lane = threadIdx.x & 63;
    const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (i >= k.n) return;   // uniform per wave
    double t[3];
    recip_grad_wave<PC>(k, i, lane, grid, home, wts, dwts, t);
    if (lane == 0) {
        tq[3 * i] = t[0];
        tq[3 * i + 1] = t[1];
        tq[3 * i + 2] = t[2];
    }
}

template <int PC>
__global__ __launch_bounds__(QEQ_BLOCK) void k_adj_grad(
    KParams k, const float* __restrict__ grid, const int* __restrict__ home, const float* __restrict__ wts,
    const float* __restrict__ dwts, const int* __restrict__ rowptr, const int* __restrict__ col,
    const float4* __restrict__ pdr, const double* __restrict__ q, const double* __restrict__ a,
    const double* __restrict__ tq, const double* __restrict__ selfgrad, const double* __restrict__ forces,
    const int* __restrict__ perm, double dLdEqeq, double dLdEelec, double* __restrict__ dchi,
    double* __restrict__ dJ, double* __restrict__ dpos) {
    const int lane = threadIdx.x & 63;
    const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (i >= k.n) return;   // uniform per wave
    double ta[3];
    recip_grad_wave<PC>(k, i, lane, grid, home, wts, dwts, ta);
    const double qi = q[i], ai = a[i];
    // pair part of d(a^T E q)/dr_i
    double fr[3] = {0.0, 0.0, 0.0};
    const int e1 = rowptr[i + 1];
    for (int e = rowptr[i] + lane; e < e1; e += 64) {
        const int j = col[e];
        const float4 d = pdr[e];
        const double c = (double)d.w * (ai * q[j] + qi * a[j]);
        fr[0] += c * d.x;
        fr[1] += c * d.y;
        fr[2] += c * d.z;
    }
    fr[0] = wave_sum(fr[0]);
    fr[1] = wave_sum(fr[1]);
    fr[2] = wave_sum(fr[2]);
    if (lane != 0) return;
    double du[3];
    for (int c = 0; c < 3; ++c) {
        du[c] = ai * tq[3 * i + c] + qi * ta[c];
        if (k.self_corr) du[c] -= ai * qi * selfgrad[3 * i + c];
    }
    const double Kd[3] = {(double)k.K1, (double)k.K2, (double)k.K3};
    const int o = perm[i];
    const double de = dLdEqeq + dLdEelec;
    if (dpos) {
        for (int c = 0; c < 3; ++c) {
            double g = fr[c];
            for (int ax = 0; ax < 3; ++ax) g += Kd[ax] * k.Hinv[c * 3 + ax] * du[ax];
            // dE_elec/dr|_q = -F
            dpos[3 * o + c] = -de * forces[3 * i + c] - g;
        }
    }
    if (dchi) dchi[o] = -ai + dLdEqeq * qi;
    if (dJ) dJ[o] = -ai * qi + 0.5 * dLdEqeq * qi * qi;
}

}  // namespace

int launch_adj_rhs(qeq_plan* pl, const double* dL_dq, double dL_dEelec) {
    const int nb = nblocks(pl->kp.n);
    hipLaunchKernelGGL(k_adj_rhs, dim3(nb), dim3(QEQ_BLOCK), 0, pl->stream, pl->kp, dL_dq, pl->perm, pl->y,
                       pl->sig, pl->dinv, dL_dEelec, pl->chi_adj, pl->part);
    QEQ_HIP(hipGetLastError());
    return launch_rhs_norm(pl, pl->chi_adj);
}

int launch_adj_gradients(qeq_plan* pl, double dL_dEqeq, double dL_dEelec, double* dL_dchi,
                         double* dL_dJ, double* dL_dpos) {
    const KParams& k = pl->kp;
    const int nbw = (k.n + QEQ_BLOCK / 64 - 1) / (QEQ_BLOCK / 64);
    // potential of q, then its gradient weights
    QEQ_TRY(launch_mesh_potential(pl, pl->q, nullptr));
    if (k.p == 6)
        hipLaunchKernelGGL((k_grad_recip<6>), dim3(nbw), dim3(QEQ_BLOCK), 0, pl->stream, k, pl->grid_r, pl->home,
                           pl->wts, pl->dwts, pl->tq);
    else
        hipLaunchKernelGGL((k_grad_recip<0>), dim3(nbw), dim3(QEQ_BLOCK), 0, pl->stream, k, pl->grid_r, pl->home,
                           pl->wts, pl->dwts, pl->tq);
    QEQ_HIP(hipGetLastError());
    // potential of a, then the combined gradient
    QEQ_TRY(launch_mesh_potential(pl, pl->q_adj, nullptr));
#define ADJ_ARGS                                                                                   \
    dim3(nbw), dim3(QEQ_BLOCK), 0, pl->stream, k, pl->grid_r, pl->home, pl->wts, pl->dwts, pl->rowptr, \
        pl->col, pl->pdr, pl->q, pl->q_adj, pl->tq, pl->selfgrad, pl->forces_s, pl->perm, dL_dEqeq,     \
        dL_dEelec, dL_dchi, dL_dJ, dL_dpos
    if (k.p == 6)
        hipLaunchKernelGGL((k_adj_grad<6>), ADJ_ARGS);
    else
        hipLaunchKernelGGL((k_adj_grad<0>), ADJ_ARGS);
#undef ADJ_ARGS
    return qeq_check(hipGetLastError());
}
