// Stabilised quasi-Newton minimisation (SQNM) of the QEq energy, the
// alternative to conjugate gradients in the paper's solver comparison
// ("Electrostatics Solvers" benchmarks): minimise
//
//     f(q) = 1/2 q^T A q + chi_eff^T q      on sum(q) = Q_tot,
//
// A = E + diag(J) (eq. 4G_qeq_prime), following the published stabilised
// quasi-Newton scheme (Schaefer, Mohr, Amsler, Goedecker 2015) in the Jacobi
// metric (coordinates z = D^{1/2} q, D_i = J_i + 1/(sigma_i sqrt(pi))):
//
//   * history: the last m displacements s_i and gradient differences y_i;
//     the overlap <s_i, s_j>_D keeps its well-conditioned eigen-subspace
//     (eigenvalues above 1e-4 of the largest), an orthonormal basis d_k;
//   * Hessian in that subspace H_kl = (d_k . dg_l + d_l . dg_k) / 2, its
//     eigenpairs (kappa_j, Ritz vectors h_j), residuals
//     |dg(h_j) - kappa_j D h_j|_{D^-1} (constraint direction removed) and
//     curvatures kappa_j' = sqrt(kappa_j^2 + res_j^2);
//   * step dq = -alpha (zJ - sum c_j h_j) - sum c_j / kappa_j' h_j with
//     c_j = h_j . (g - c0 1), zJ = D^-1 (g - c0 1), c0 = sum D^-1 g / sum D^-1,
//     projected back onto the plane;
//   * an energy rise undoes the step, halves alpha and clears the history;
//     otherwise alpha grows by 5% when consecutive projected gradients
//     still point the same way (cosine > 0.2) and halves when they point
//     against each other (cosine < 0).
//
// On the GPU every n-vector operation is a kernel over the sorted atoms
// (FP64 vectors; the operator product is the solve's FP32 mesh/pair path);
// one pass collects every dot product the host needs (overlaps, s.y, y.y in
// the D^-1 metric, sums, energy terms) into block partials, one kernel
// reduces them, and the host does the m x m eigenproblems and sends the step
// coefficients back as kernel arguments: one host sync per iteration.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "internal.h"

namespace {

constexpr int SQ_MAX_M = 16;              // history length limit
constexpr int SQ_MAX_H = SQ_MAX_M + 1;    // slots: history plus the trial pair
constexpr int SQ_NS_MAX = 3 * SQ_MAX_H * SQ_MAX_H + 3 * SQ_MAX_H + 16;   // descriptors at most
constexpr int SQ_NT = 256;
constexpr int SQ_CHUNK = 128;             // atoms staged per block
constexpr double SQ_EPS_SIG = 1e-4;
// The gradient comes from the FP32 operator: its relative residual has a
// floor near 1e-7 (the CG path accepts a true residual up to 2 max(tol, 1e-7)
// for the same reason), and energy differences below ~1e-6 of the energy's
// terms are rounding, not rises.
constexpr double SQ_RES_FLOOR = 1e-7;
constexpr double SQ_F_NOISE = 1e-6;

// weights of a descriptor: none, D (= 1 / D^-1), D^-1
enum SqWeight { SQ_W1 = 0, SQ_WD = 1, SQ_WDINV = 2 };

struct SqSlots {
    int h;                    // history vectors staged (0 .. SQ_MAX_H)
    int slot[SQ_MAX_H];       // ring slots of s_i / y_i
};

struct SqStep {
    int h;
    int slot[SQ_MAX_M];
    double a[SQ_MAX_M];       // coefficients of the history displacements
    double b;                 // coefficient of zJ = D^-1 (g - c0)
    double c0;
    double corr;              // coefficient of D^-1 (back onto the plane)
    int out;                  // ring slot that receives the step
};

// x += dq, dq = sum a_j s_j + b D^-1 (g - c0) + corr D^-1, stored in slot out.
__global__ __launch_bounds__(SQ_NT) void k_sq_step(int n, int ld, SqStep st, const double* __restrict__ S,
                                                 const double* __restrict__ g, const double* __restrict__ dinv,
                                                 double* __restrict__ x, double* __restrict__ Sout) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double di = dinv[i];
    double d = di * (st.b * (g[i] - st.c0) + st.corr);
    for (int j = 0; j < st.h; ++j) d += st.a[j] * S[(size_t)st.slot[j] * ld + i];
    Sout[i] = d;
    x[i] += d;
}

// x -= s (an undone step)
__global__ __launch_bounds__(SQ_NT) void k_sq_undo(int n, const double* __restrict__ s, double* __restrict__ x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] -= s[i];
}

// g = E x + J x + chi_eff; with yout also y = g - g_prev.
__global__ __launch_bounds__(SQ_NT) void k_sq_grad(int n, const double* __restrict__ x,
                                                 const double* __restrict__ ex, const double* __restrict__ Jv,
                                                 const double* __restrict__ chi, const double* __restrict__ gprev,
                                                 double* __restrict__ g, double* __restrict__ yout) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double gi = ex[i] + Jv[i] * x[i] + chi[i];
    g[i] = gi;
    if (yout) yout[i] = gi - gprev[i];
}

// Block partials of the descriptor list over a chunk of SQ_CHUNK atoms,
// staged in LDS as vectors: s_0..s_{h-1}, y_0..y_{h-1}, g, g_prev, x, chi,
// D^-1, 1.  A descriptor names two staged vectors u, w and a weight (none,
// D, D^-1): its sum is sum_a u_a w_a weight_a.
__global__ __launch_bounds__(SQ_NT) void k_sq_sums(int n, int ld, SqSlots sl, int ns, const int* __restrict__ desc,
                                                 const double* __restrict__ S, const double* __restrict__ Y,
                                                 const double* __restrict__ g, const double* __restrict__ gprev,
                                                 const double* __restrict__ x, const double* __restrict__ chi,
                                                 const double* __restrict__ dinv, double* __restrict__ part) {
    extern __shared__ double sq_sm[];
    const int a0 = blockIdx.x * SQ_CHUNK;
    const int na = min(SQ_CHUNK, n - a0);
    const int h = sl.h;
    const int nv = 2 * h + 6;
    for (int t = threadIdx.x; t < nv * SQ_CHUNK; t += SQ_NT) {
        const int v = t / SQ_CHUNK, a = t - v * SQ_CHUNK;
        double val = 0.0;
        if (a < na) {
            const int i = a0 + a;
            if (v < h) val = S[(size_t)sl.slot[v] * ld + i];
            else if (v < 2 * h) val = Y[(size_t)sl.slot[v - h] * ld + i];
            else if (v == 2 * h) val = g[i];
            else if (v == 2 * h + 1) val = gprev ? gprev[i] : 0.0;
            else if (v == 2 * h + 2) val = x[i];
            else if (v == 2 * h + 3) val = chi[i];
            else if (v == 2 * h + 4) val = dinv[i];
            else val = 1.0;
        }
        sq_sm[t] = val;
    }
    __syncthreads();
    const double* dv = sq_sm + (size_t)(2 * h + 4) * SQ_CHUNK;
    for (int p = threadIdx.x; p < ns; p += SQ_NT) {
        const int dsc = desc[p];
        const int wk = dsc >> 16, iu = (dsc >> 8) & 255, iw = dsc & 255;
        const double* u = sq_sm + (size_t)iu * SQ_CHUNK;
        const double* w = sq_sm + (size_t)iw * SQ_CHUNK;
        double acc = 0.0;
        if (wk == 0) {
            for (int a = 0; a < na; ++a) acc += u[a] * w[a];
        } else if (wk == 1) {
            for (int a = 0; a < na; ++a) acc += u[a] * w[a] / dv[a];
        } else {
            for (int a = 0; a < na; ++a) acc += u[a] * w[a] * dv[a];
        }
        part[(size_t)blockIdx.x * ns + p] = acc;
    }
}

__global__ __launch_bounds__(SQ_NT) void k_sq_reduce(int nb, int ns, const double* __restrict__ part,
                                                   double* __restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ns) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(size_t)b * ns + p];
    out[p] = s;
}

// ---------------------------------------------------------------- host side

// Symmetric eigenproblem by cyclic Jacobi rotations (n <= SQ_MAX_H):
// a (row-major, destroyed) -> eigenvalues w, eigenvectors as columns of v.
void jacobi_eig(int n, std::vector<double>& a, std::vector<double>& w, std::vector<double>& v) {
    v.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += a[(size_t)i * n + j] * a[(size_t)i * n + j];
                if (i != j) off += a[(size_t)i * n + j] * a[(size_t)i * n + j];
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = a[(size_t)p * n + q];
                if (fabs(apq) < 1e-300) continue;
                const double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
                const double theta = 0.5 * (aqq - app) / apq;
                const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
                    a[(size_t)k * n + p] = c * akp - s * akq;
                    a[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
                    a[(size_t)p * n + k] = c * apk - s * aqk;
                    a[(size_t)q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
                    v[(size_t)k * n + p] = c * vkp - s * vkq;
                    v[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = a[(size_t)i * n + i];
}

int pack(int weight, int u, int w) { return (weight << 16) | (u << 8) | w; }

// Descriptor list for h staged history vectors and index tables into it.
// Staged vector numbers: s_i = i, y_i = h + i, g = 2h, g_prev = 2h + 1,
// x = 2h + 2, chi = 2h + 3, D^-1 = 2h + 4, 1 = 2h + 5.
struct SqLayout {
    int h = 0, ns = 0;
    int sds[SQ_MAX_H][SQ_MAX_H], sy[SQ_MAX_H][SQ_MAX_H], ydy[SQ_MAX_H][SQ_MAX_H];
    int dy[SQ_MAX_H], ssum[SQ_MAX_H], sg[SQ_MAX_H];
    int gsum, g2, dg, xg, cx, dgg, dg2;
    std::vector<int> desc;
    void build(int hh) {
        h = hh;
        desc.clear();
        const int G = 2 * h, GP = 2 * h + 1, X = 2 * h + 2, CHI = 2 * h + 3, ONE = 2 * h + 5;
        auto add = [&](int weight, int u, int w) {
            desc.push_back(pack(weight, u, w));
            return (int)desc.size() - 1;
        };
        for (int i = 0; i < h; ++i)
            for (int j = i; j < h; ++j) sds[i][j] = sds[j][i] = add(SQ_WD, i, j);
        for (int i = 0; i < h; ++i)
            for (int j = 0; j < h; ++j) sy[i][j] = add(SQ_W1, i, h + j);
        for (int i = 0; i < h; ++i)
            for (int j = i; j < h; ++j) ydy[i][j] = ydy[j][i] = add(SQ_WDINV, h + i, h + j);
        for (int i = 0; i < h; ++i) {
            dy[i] = add(SQ_WDINV, h + i, ONE);
            ssum[i] = add(SQ_W1, i, ONE);
            sg[i] = add(SQ_W1, i, G);
        }
        gsum = add(SQ_W1, G, ONE);
        g2 = add(SQ_W1, G, G);
        dg = add(SQ_WDINV, G, ONE);
        xg = add(SQ_W1, X, G);      // x . g; x . A x = x . g - chi . x
        cx = add(SQ_W1, CHI, X);
        dgg = add(SQ_WDINV, G, GP);
        dg2 = add(SQ_WDINV, G, G);
        ns = (int)desc.size();
    }
};

template <typename T>
int sq_alloc(T** p, size_t count) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    if (hipMalloc((void**)p, sizeof(T) * (count ? count : 1)) != hipSuccess) return QEQ_ENOMEM;
    if (poisonable<T>) debug_poison(*p, sizeof(T) * count);
    return QEQ_OK;
}

int sq_buffers(qeq_plan* pl) {
    const int m = pl->sq_m;
    if (pl->sq_cap_n >= pl->n_max && pl->sq_cap_m >= m) return QEQ_OK;
    const size_t nn = (size_t)pl->n_max;
    QEQ_TRY(sq_alloc(&pl->sq_S, (size_t)(m + 1) * nn));
    QEQ_TRY(sq_alloc(&pl->sq_Y, (size_t)(m + 1) * nn));
    QEQ_TRY(sq_alloc(&pl->sq_g, 2 * nn));
    QEQ_TRY(sq_alloc(&pl->sq_part, (size_t)((nn + SQ_CHUNK - 1) / SQ_CHUNK) * SQ_NS_MAX));
    QEQ_TRY(sq_alloc(&pl->sq_sums, (size_t)SQ_NS_MAX));
    QEQ_TRY(sq_alloc(&pl->sq_desc, (size_t)SQ_NS_MAX));
    if (!pl->sq_host) {
        if (hipHostMalloc((void**)&pl->sq_host, sizeof(double) * SQ_NS_MAX, hipHostMallocDefault) != hipSuccess) {
            pl->sq_host = nullptr;
            return QEQ_ENOMEM;
        }
    }
    pl->sq_cap_n = pl->n_max;
    pl->sq_cap_m = m;
    return QEQ_OK;
}

// Sums over the staged history (ring slots in order), g = sq_g[gi], g_prev.
int sq_collect(qeq_plan* pl, SqLayout& L, const std::vector<int>& slots, const double* g, const double* gprev) {
    const int n = pl->kp.n;
    L.build((int)slots.size());
    QEQ_HIP(hipMemcpyAsync(pl->sq_desc, L.desc.data(), sizeof(int) * L.ns, hipMemcpyHostToDevice, pl->stream));
    SqSlots sl{};
    sl.h = (int)slots.size();
    for (int i = 0; i < sl.h; ++i) sl.slot[i] = slots[i];
    const int nb = (n + SQ_CHUNK - 1) / SQ_CHUNK;
    const size_t sh = sizeof(double) * (size_t)(2 * sl.h + 6) * SQ_CHUNK;
    if (sh > 65536)
        QEQ_HIP(hipFuncSetAttribute((const void*)k_sq_sums, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));
    hipLaunchKernelGGL(k_sq_sums, dim3(nb), dim3(SQ_NT), sh, pl->stream, n, pl->n_max, sl, L.ns, pl->sq_desc,
                       pl->sq_S, pl->sq_Y, g, gprev, pl->q, pl->chi, pl->dinv, pl->sq_part);
    hipLaunchKernelGGL(k_sq_reduce, dim3((L.ns + SQ_NT - 1) / SQ_NT), dim3(SQ_NT), 0, pl->stream, nb, L.ns,
                       pl->sq_part, pl->sq_sums);
    QEQ_TRY(qeq_check(hipGetLastError()));
    QEQ_HIP(hipMemcpyAsync(pl->sq_host, pl->sq_sums, sizeof(double) * L.ns, hipMemcpyDeviceToHost, pl->stream));
    QEQ_HIP(hipStreamSynchronize(pl->stream));   // the descriptor vector and the sums
    return QEQ_OK;
}

// Step coefficients from the sums of the staged history (first `hist`
// entries of the layout) and the current gradient.
void sq_coefficients(const SqLayout& L, const double* v, int hist, const std::vector<int>& slots, double alpha,
                     double dinv_sum, SqStep& st) {
    const double c0 = v[L.dg] / dinv_sum;
    st.h = hist;
    st.b = -alpha;
    st.c0 = c0;
    for (int i = 0; i < hist; ++i) {
        st.slot[i] = slots[i];
        st.a[i] = 0.0;
    }
    double step_sum = -alpha * (v[L.dg] - c0 * dinv_sum);   // sum zJ (zero up to rounding)
    if (hist > 0) {
        const int h = hist;
        std::vector<double> nrm(h), ov((size_t)h * h), lam, V;
        for (int i = 0; i < h; ++i) nrm[i] = sqrt(std::max(v[L.sds[i][i]], 1e-300));
        for (int i = 0; i < h; ++i)
            for (int j = 0; j < h; ++j) ov[(size_t)i * h + j] = v[L.sds[i][j]] / (nrm[i] * nrm[j]);
        jacobi_eig(h, ov, lam, V);
        double lmax = 0.0;
        for (double l : lam) lmax = std::max(lmax, l);
        // Bs: coefficients of the orthonormal basis d_k in the raw s_i
        std::vector<double> Bs;
        int nk = 0;
        for (int k = 0; k < h; ++k) {
            if (!(lam[k] > SQ_EPS_SIG * lmax)) continue;
            for (int i = 0; i < h; ++i) Bs.push_back(V[(size_t)i * h + k] / (sqrt(lam[k]) * nrm[i]));
            ++nk;
        }
        auto B = [&](int i, int k) { return Bs[(size_t)k * h + i]; };
        // subspace Hessian
        std::vector<double> H((size_t)nk * nk), kap, U;
        for (int k = 0; k < nk; ++k)
            for (int l = 0; l < nk; ++l) {
                double t = 0.0;
                for (int i = 0; i < h; ++i)
                    for (int j = 0; j < h; ++j)
                        t += B(i, k) * B(j, l) * 0.5 * (v[L.sy[i][j]] + v[L.sy[j][i]]);
                H[(size_t)k * nk + l] = t;
            }
        jacobi_eig(nk, H, kap, U);
        for (int jr = 0; jr < nk; ++jr) {
            // Ritz vector h = sum_i C_i s_i
            std::vector<double> C(h, 0.0);
            for (int i = 0; i < h; ++i)
                for (int k = 0; k < nk; ++k) C[i] += B(i, k) * U[(size_t)k * nk + jr];
            double rDr = 0.0, rh = 0.0, hDh = 0.0, Dr = 0.0, hs = 0.0, hg = 0.0;
            for (int i = 0; i < h; ++i) {
                Dr += C[i] * v[L.dy[i]];
                hs += C[i] * v[L.ssum[i]];
                hg += C[i] * v[L.sg[i]];
                for (int j = 0; j < h; ++j) {
                    rDr += C[i] * C[j] * v[L.ydy[i][j]];
                    rh += C[i] * C[j] * v[L.sy[j][i]];   // y_i . s_j
                    hDh += C[i] * C[j] * v[L.sds[i][j]];
                }
            }
            const double kj = kap[jr];
            // |r - kappa D h - c 1|^2 in the D^-1 metric, c = sum D^-1 (r - kappa D h) / sum D^-1
            const double c = (Dr - kj * hs) / dinv_sum;
            double rn2 = rDr - 2.0 * kj * rh + kj * kj * hDh - 2.0 * c * (Dr - kj * hs) + c * c * dinv_sum;
            rn2 = std::max(rn2, 0.0);
            const double ks = sqrt(kj * kj + rn2);
            const double cj = hg - c0 * hs;
            const double coef = (alpha - (ks > 0.0 ? 1.0 / ks : 0.0)) * cj;
            for (int i = 0; i < h; ++i) st.a[i] += coef * C[i];
        }
        for (int i = 0; i < h; ++i) step_sum += st.a[i] * v[L.ssum[i]];
    }
    st.corr = -step_sum / dinv_sum;
}

}  // namespace

void sqnm_free(qeq_plan* pl) {
    void* ptrs[] = {pl->sq_S, pl->sq_Y, pl->sq_g, pl->sq_part, pl->sq_sums, pl->sq_desc};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    if (pl->sq_host) (void)hipHostFree(pl->sq_host);
    pl->sq_S = pl->sq_Y = pl->sq_g = pl->sq_part = pl->sq_sums = nullptr;
    pl->sq_desc = nullptr;
    pl->sq_host = nullptr;
    pl->sq_cap_n = pl->sq_cap_m = 0;
}

// SQNM from q0 (or Q/N) on the plan's current operator (periodic: mesh,
// Ewald sums or Gaussian-on-grid), then the final pass of the CG path.
int sqnm_run(qeq_plan* pl, const double* q0, double* q_out, double* energies, double* forces_out, bool* conv_out) {
    QEQ_TRY(sq_buffers(pl));
    const int n = pl->kp.n, m = pl->sq_m, ld = pl->n_max;
    const int nb = nblocks(n, SQ_NT);
    pl->warm_rejected = false;
    QEQ_TRY(launch_cg_init_q(pl, q0));   // q on the plane; clears the CG flags
    QEQ_HIP(hipMemcpyAsync(pl->sc_host, pl->sc, sizeof(CgScalars), hipMemcpyDeviceToHost, pl->stream));
    QEQ_HIP(hipStreamSynchronize(pl->stream));
    const double chi_norm = pl->sc_host->chi_norm > 0.0 ? pl->sc_host->chi_norm : 1.0;
    const double dinv_sum = pl->sc_host->dinv_sum;
    double* gbuf[2] = {pl->sq_g, pl->sq_g + ld};
    int gcur = 0;
    // gradient and sums at the start
    QEQ_TRY(operator_product(pl, pl->q, pl->y));
    hipLaunchKernelGGL(k_sq_grad, dim3(nb), dim3(SQ_NT), 0, pl->stream, n, pl->q, pl->y, pl->Jv, pl->chi,
                       nullptr, gbuf[gcur], nullptr);
    SqLayout L;
    std::vector<int> hist;   // ring slots, oldest first
    QEQ_TRY(sq_collect(pl, L, hist, gbuf[gcur], nullptr));
    std::vector<double> v(pl->sq_host, pl->sq_host + L.ns);
    // f = 1/2 x.A x + chi.x with x.A x = x.g - chi.x
    auto energy = [&](const std::vector<double>& s, const SqLayout& l) { return 0.5 * (s[l.xg] - s[l.cx]) + s[l.cx]; };
    auto resid = [&](const std::vector<double>& s, const SqLayout& l) {
        return sqrt(std::max(s[l.g2] - s[l.gsum] * s[l.gsum] / n, 0.0)) / chi_norm;
    };
    double f = energy(v, L), res = resid(v, L);
    double dg_cur = v[L.dg], dg2_cur = v[L.dg2];
    double alpha = 1.0;
    int it = 0, rejected = 0;
    const double tol = std::max(pl->prm.tol, SQ_RES_FLOOR);
    SqStep st{};
    std::vector<int> free_slots;
    for (int s = m; s >= 0; --s) free_slots.push_back(s);
    while (res > tol && it < pl->prm.max_iter) {
        ++it;
        // step from the current history and gradient
        sq_coefficients(L, v.data(), (int)hist.size(), hist, alpha, dinv_sum, st);
        st.out = free_slots.back();
        hipLaunchKernelGGL(k_sq_step, dim3(nb), dim3(SQ_NT), 0, pl->stream, n, ld, st, pl->sq_S, gbuf[gcur],
                           pl->dinv, pl->q, pl->sq_S + (size_t)st.out * ld);
        QEQ_TRY(qeq_check(hipGetLastError()));
        // trial gradient and the trial pair (s, y) in slot st.out
        QEQ_TRY(operator_product(pl, pl->q, pl->y));
        hipLaunchKernelGGL(k_sq_grad, dim3(nb), dim3(SQ_NT), 0, pl->stream, n, pl->q, pl->y, pl->Jv, pl->chi,
                           gbuf[gcur], gbuf[gcur ^ 1], pl->sq_Y + (size_t)st.out * ld);
        std::vector<int> staged = hist;
        staged.push_back(st.out);
        if ((int)staged.size() > m) staged.erase(staged.begin());
        SqLayout Lt;
        QEQ_TRY(sq_collect(pl, Lt, staged, gbuf[gcur ^ 1], gbuf[gcur]));
        std::vector<double> vt(pl->sq_host, pl->sq_host + Lt.ns);
        const double f_new = energy(vt, Lt), res_new = resid(vt, Lt);
        const double f_noise = SQ_F_NOISE * (0.5 * fabs(vt[Lt.xg] - vt[Lt.cx]) + fabs(vt[Lt.cx]));
        if (f_new > f + f_noise && res_new > tol) {
            // energy rose: undo, shorter steps, fresh history
            hipLaunchKernelGGL(k_sq_undo, dim3(nb), dim3(SQ_NT), 0, pl->stream, n, pl->sq_S + (size_t)st.out * ld,
                               pl->q);
            QEQ_TRY(qeq_check(hipGetLastError()));
            alpha *= 0.5;
            ++rejected;
            if (alpha < 1e-12) break;   // no descent left at this precision
            for (int s : hist) free_slots.push_back(s);
            hist.clear();
            // the layout of an empty history from the kept scalars
            L.build(0);
            v.assign(L.ns, 0.0);
            v[L.dg] = dg_cur;
            v[L.dg2] = dg2_cur;
            continue;
        }
        // accepted: the trial pair joins the history
        free_slots.pop_back();
        if ((int)hist.size() + 1 > m) {
            free_slots.push_back(hist.front());
            hist.erase(hist.begin());
        }
        hist.push_back(st.out);
        // gradient feedback on alpha: cosine of consecutive projected gradients (D^-1 metric)
        const double c_new = vt[Lt.dg] / dinv_sum, c_old = dg_cur / dinv_sum;
        const double cross = vt[Lt.dgg] - c_old * vt[Lt.dg] - c_new * dg_cur + c_new * c_old * dinv_sum;
        const double nn = vt[Lt.dg2] - c_new * vt[Lt.dg];
        const double no = dg2_cur - c_old * dg_cur;
        const double cosv = cross / sqrt(std::max(nn * no, 1e-300));
        if (cosv > 0.2) alpha *= 1.05;
        else if (cosv < 0.0) alpha *= 0.5;
        gcur ^= 1;
        f = f_new;
        res = res_new;
        dg_cur = vt[Lt.dg];
        dg2_cur = vt[Lt.dg2];
        L = Lt;
        v.swap(vt);
    }
    pl->sq_iters = it;
    pl->sq_rejected = rejected;
    const bool conv = res <= tol || res <= 2.0 * std::max(pl->prm.tol, SQ_RES_FLOOR);
    // the CG scalars the final pass and the status read
    QEQ_HIP(hipMemcpyAsync(&pl->sc->iters, &it, sizeof(int), hipMemcpyHostToDevice, pl->stream));
    QEQ_HIP(hipMemcpyAsync(&pl->sc->res, &res, sizeof(double), hipMemcpyHostToDevice, pl->stream));
    QEQ_TRY(final_pass(pl, q_out, energies, forces_out));
    *conv_out = conv;
    return QEQ_OK;
}
