// Element-resolved electrostatic potentials: the embedding features of the
// paper's ee4G variant (Electrostatics and Charge Equilibration section: a
// vector of element-specific potentials at each site, computed from the
// equilibrated charges, appended to the atomic feature vectors).
//
//   Gamma_i^z = sum_j E_ij q_j [s_j = z] - [s_i = z] q_i / (sigma_i sqrt(pi)),
//
// the potential at atom i of the charges of element z without the atom's own
// Gaussian self term, with E the Coulomb operator of the last solve on the
// plan (periodic: particle mesh + real-space pairs + self + background;
// isolated: the direct pair sum).  One operator product per element, with
// the element's charges as the source; the tape of the solve is left intact.
#include <math.h>

#include "internal.h"

namespace {

constexpr double EMB_RSQPI = 0.56418958354775628695;   // 1/sqrt(pi)

// v[i] = q_i [s_i = z] in caller order, from the solve's sorted charges.
__global__ void k_elem_src(int n, int z, const double* __restrict__ q_s, const int* __restrict__ perm,
                           const int32_t* __restrict__ species, double* __restrict__ v) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int i = perm[s];
    v[i] = species[i] == z ? q_s[s] : 0.0;
}

// out[i][z] = w[i] - [s_i = z] q_i / (sigma_i sqrt(pi)), caller order.
__global__ void k_elem_out(int n, int z, int n_elem, const double* __restrict__ w, const double* __restrict__ q_s,
                           const double* __restrict__ sig_s, const int* __restrict__ perm,
                           const int32_t* __restrict__ species, double* __restrict__ out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int i = perm[s];
    const double self = species[i] == z ? q_s[s] * EMB_RSQPI / sig_s[s] : 0.0;
    out[(size_t)i * n_elem + z] = w[i] - self;
}

}  // namespace

int element_potentials_impl(qeq_plan* pl, const int32_t* species, int n_elem, double* out) {
    if (!species || !out || n_elem < 1 || n_elem > QEQ_MAX_ELEMENTS) return QEQ_EINVAL;
    const bool periodic = pl->tape_valid && !pl->direct;
    const bool isolated = pl->direct && pl->np_valid;
    if (!periodic && !isolated) return QEQ_EINVAL;
    if (!pl->elem_buf) {
        if (hipMalloc((void**)&pl->elem_buf, sizeof(double) * 2 * (size_t)pl->n_max) != hipSuccess) {
            pl->elem_buf = nullptr;
            return QEQ_ENOMEM;
        }
        debug_poison(pl->elem_buf, sizeof(double) * 2 * (size_t)pl->n_max);
    }
    const int n = pl->kp.n;
    const int nb = nblocks(n);
    double* v = pl->elem_buf;
    double* w = pl->elem_buf + pl->n_max;
    // the solve's E q (pl->y) belongs to the tape: products go to the
    // adjoint's scratch vector instead
    std::swap(pl->y, pl->y_adj);
    int rc = QEQ_OK;
    for (int z = 0; z < n_elem && rc == QEQ_OK; ++z) {
        hipLaunchKernelGGL(k_elem_src, dim3(nb), dim3(QEQ_BLOCK), 0, pl->stream, n, z, pl->q, pl->perm, species, v);
        rc = qeq_check(hipGetLastError());
        if (rc == QEQ_OK) {
            if (isolated) {
                rc = launch_np_matvec(pl, v, w, QEQ_MODE_ELEC);
            } else {
                rc = launch_matvec_io(pl, v, nullptr, 0);
                if (rc == QEQ_OK) rc = launch_mesh_potential(pl, pl->pvec, nullptr);
                if (rc == QEQ_OK) rc = launch_interp(pl, pl->pvec, pl->y, QEQ_MODE_MATVEC, 0);
                if (rc == QEQ_OK) rc = launch_matvec_io(pl, nullptr, w, 1);
            }
        }
        if (rc == QEQ_OK) {
            hipLaunchKernelGGL(k_elem_out, dim3(nb), dim3(QEQ_BLOCK), 0, pl->stream, n, z, n_elem, w, pl->q,
                               pl->sig, pl->perm, species, out);
            rc = qeq_check(hipGetLastError());
        }
    }
    std::swap(pl->y, pl->y_adj);
    return rc;
}
