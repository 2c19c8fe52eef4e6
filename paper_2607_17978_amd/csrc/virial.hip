// Virial of the electrostatic energy at the solution charges (SI, "Stress
// Tensor": sigma = (1/V) dE/d eps; an MD code takes the virial -V sigma).
//
// W_ab = -dE_elec/d eps_ab under the homogeneous strain r -> (1 + eps) r of
// positions and lattice vectors (fractional coordinates fixed).  At the QEq
// solution this is also -dE_QEq/d eps: E_QEq is stationary in q on the plane
// sum(q) = Q, and J and chi do not depend on the geometry.  The Electrostatics
// Solvers section obtains the stress from the same Fourier machinery as the
// forces; here every term of the discretised energy is differentiated:
//
//   mesh        E = 1/2 sum_m G(m) |Q(m)|^2 with Q(m) fixed (fractional
//               coordinates), G's strain factor -delta + 2 (1/k^2 + eta^2/2) k k
//               -> W = 1/2 sum_m G |Q|^2 (delta - 2 (1/k^2 + eta^2/2) k k);
//   real space  1/2 sum_ij q_i q_j K(r_ij) -> W = -1/2 sum q_i q_j K'(r)/r d d;
//   self corr.  1/2 sum q_i^2 (C_eta - theta_i^T Theta theta_i)
//               -> W = -1/2 sum q_i^2 (dC_eta - theta_i^T dTheta theta_i);
//   background  E_bg = -(pi/V)(eta^2 Q^2 - 2 Q sum q sigma^2) ~ 1/V -> W = E_bg delta;
//   Gaussian self energies: no length, no term.
#include <math.h>

#include "internal.h"

namespace {

constexpr double PI = 3.14159265358979323846;

int alloc_doubles(double** p, size_t count) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    if (hipMalloc((void**)p, sizeof(double) * count) != hipSuccess) return QEQ_ENOMEM;
    debug_poison(*p, sizeof(double) * count);
    return QEQ_OK;
}

// Real-space pair virial: one wave per atom over its CSR row (pairs are
// stored in both directions, hence the 1/2 at the end).  pdr holds
// (r_i - r_j(image), K'(r)/r).
__global__ __launch_bounds__(QEQ_BLOCK) void k_virial_pairs(KParams k, const double* __restrict__ q,
                                                           const int* __restrict__ rowptr,
                                                           const int* __restrict__ col,
                                                           const float4* __restrict__ pdr,
                                                           double* __restrict__ part) {
    const int lane = threadIdx.x & 63;
    const int nwaves = gridDim.x * (blockDim.x >> 6);
    double acc[QEQ_NPART];
#pragma unroll
    for (int t = 0; t < QEQ_NPART; ++t) acc[t] = 0.0;
    for (int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < k.n; i += nwaves) {
        double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        const int e1 = rowptr[i + 1];
        for (int e = rowptr[i] + lane; e < e1; e += 64) {
            const float4 d = pdr[e];
            const double c = (double)d.w * q[col[e]];
            const double dx = d.x, dy = d.y, dz = d.z;
            v[0] += c * dx * dx;
            v[1] += c * dy * dy;
            v[2] += c * dz * dz;
            v[3] += c * dx * dy;
            v[4] += c * dx * dz;
            v[5] += c * dy * dz;
        }
        const double qi = q[i];
#pragma unroll
        for (int t = 0; t < 6; ++t) acc[t] += qi * v[t];
    }
    block_sum<QEQ_NPART>(acc);
    if (threadIdx.x == 0)
        for (int t = 0; t < QEQ_NPART; ++t) part[(size_t)blockIdx.x * QEQ_NPART + t] = acc[t];
}

// Sums the three sets of partials and writes W (row-major 3 x 3).
//   mesh  [sum e, sum e c k_a k_b (6)]
//   pairs [sum q_i q_j K'/r d_a d_b (6)]
//   self  [sum q^2 theta^T dTheta_ab theta (6), sum q^2, sum q sigma^2]
__global__ void k_virial_finish(KParams k, const double* __restrict__ pm, int nm, const double* __restrict__ pp,
                                int np, const double* __restrict__ ps, int ns, double dc0, double dc1,
                                double dc2, double dc3, double dc4, double dc5, double* __restrict__ out) {
    double tm[QEQ_NPART], tp[QEQ_NPART], ts[QEQ_NPART];
    reduce_partials<QEQ_NPART>(pm, nm, tm);
    reduce_partials<QEQ_NPART>(pp, np, tp);
    reduce_partials<QEQ_NPART>(ps, ns, ts);
    if (threadIdx.x != 0) return;
    const double dc[6] = {dc0, dc1, dc2, dc3, dc4, dc5};
    const double qt = k.q_tot;
    const double e_bg = -(PI / k.vol) * (k.eta * k.eta * qt * qt - 2.0 * qt * ts[7]);
    double w[6];
    for (int c = 0; c < 6; ++c) {
        const double diag = c < 3 ? 1.0 : 0.0;
        double v = 0.5 * (tm[0] * diag - tm[1 + c]);   // mesh
        v -= 0.5 * tp[c];                              // real space
        if (k.self_corr) v -= 0.5 * (dc[c] * ts[6] - ts[c]);
        v += e_bg * diag;
        w[c] = v;
    }
    out[0] = w[0];
    out[4] = w[1];
    out[8] = w[2];
    out[1] = out[3] = w[3];
    out[2] = out[6] = w[4];
    out[5] = out[7] = w[5];
}

}  // namespace

int virial_impl(qeq_plan* pl, double* virial) {
    if (!pl->tape_valid || !virial) return QEQ_EINVAL;
    const KParams& k = pl->kp;
    const int nm = mesh_virial_blocks(k);
    const int np = std::min(4096, (k.n + QEQ_BLOCK / 64 - 1) / (QEQ_BLOCK / 64));
    const int ns = nblocks(k.n);
    const size_t need = (size_t)(nm + np + ns) * QEQ_NPART;
    if (need > pl->vir_cap) {
        pl->vir_cap = 0;
        QEQ_TRY(alloc_doubles(&pl->vir_part, need));
        pl->vir_cap = need;
    }
    double* pm = pl->vir_part;
    double* pp = pm + (size_t)nm * QEQ_NPART;
    double* ps = pp + (size_t)np * QEQ_NPART;
    if (k.self_corr && !pl->strain_valid) {
        if (!pl->strain_tab) {
            const int np1 = 2 * QEQ_MAXP - 1;
            QEQ_TRY(alloc_doubles(&pl->strain_tab, (size_t)6 * np1 * np1 * np1));
        }
        reciprocal_self_strain(k.H, k.Hinv, k.vol, k.eta, pl->dc_eta);
        QEQ_TRY(launch_theta_strain(pl, pl->strain_tab));
        pl->strain_valid = true;
    }
    QEQ_TRY(launch_mesh_virial(pl, pl->q, pm));
    hipLaunchKernelGGL(k_virial_pairs, dim3(np), dim3(QEQ_BLOCK), 0, pl->stream, k, pl->q, pl->rowptr, pl->col,
                       pl->pdr, pp);
    QEQ_TRY(qeq_check(hipGetLastError()));
    QEQ_TRY(launch_self_strain(pl, k.self_corr ? pl->strain_tab : nullptr, ps));
    const double* dc = pl->dc_eta;
    hipLaunchKernelGGL(k_virial_finish, dim3(1), dim3(256), 0, pl->stream, k, pm, nm, pp, np, ps, ns, dc[0], dc[1],
                       dc[2], dc[3], dc[4], dc[5], virial);
    QEQ_TRY(qeq_check(hipGetLastError()));
    QEQ_HIP(hipStreamSynchronize(pl->stream));
    return QEQ_OK;
}
