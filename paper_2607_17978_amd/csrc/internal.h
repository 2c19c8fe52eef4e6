// Internal interfaces of the particle-mesh QEq library: the kernel-argument
// bundle, the plan (device workspace) and the host launchers of every kernel.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <vector>

#include "common.h"
#include "../../include/qeq.h"

#define QEQ_BLOCK 256         // threads per block for per-atom kernels
#define QEQ_VBLOCK 256        // threads per block of the CG vector kernels
#define QEQ_FFT_THREADS 256   // threads per block for FFT passes
#define QEQ_NPART 8           // doubles per block in partial-sum buffers

// Bits of the device error word.
#define QEQ_ERRBIT_INPUT 1

// Interp / final-kernel modes
#define QEQ_MODE_CG 0         // y = (E + diag J) p over the selected parts
#define QEQ_MODE_MATVEC 1     // y = E v over the selected parts (no J)
#define QEQ_MODE_FINAL 2      // y = E q, forces, energy partials
#define QEQ_MODE_ELEC 3       // direct pair sum only: y = E v (no J, no partial sums)
#define QEQ_MAX_ELEMENTS 16   // element channels of qeq_element_potentials

#define QEQ_PART_RECIP 1
#define QEQ_PART_REAL 2
#define QEQ_PART_SELF 4
#define QEQ_PART_BG 8

// Everything a kernel needs to know about the problem, passed by value.
struct KParams {
    int n;
    int p;                    // spline order
    int K1, K2, K3, K3h;      // grid; K3h = K3 / 2 + 1 (half spectrum along axis 3)
    int TW, TWlog2, ntile;    // axis-2 row tile of the C2R and axis-1 passes
    int TWS, ntile_s;         // axis-2 row tile of the spread + R2C pass
    int NR, NRlog2;           // rows per block of the axis-2 pass
    int nc[3];                // real-space cell-list dims
    int ns[3];                // stencil half-widths in cells
    int parts;                // operator parts (QEQ_PART_*)
    int self_corr;
    double H[9];              // rows = lattice vectors
    double Hinv[9];
    double M[6];              // (H H^T)^-1: 11 22 33 12 13 23
    double vol;
    double eta;
    double eta_green;         // screening width in the mesh Green's function (0: plain 4 pi / k^2)
    double rc, rc2;
    double green_pref;        // 4 pi / V
    double bg_pref;           // 2 pi / V
    double q_tot;
    double c_eta;             // (4 pi / V) sum_{k != 0} exp(-eta^2 k^2 / 2) / k^2
    double tol;
};

// Geometry of the Gaussian-on-grid (plane-wave) operator, in grid steps:
// a grid point at integer offsets t from the atom's cell, d = t - frac(u),
// lies at squared distance d^T G d from the atom.
struct PwGeom {
    float G[6];       // (a_a . a_b) / (K_a K_b): 11 22 33 12 13 23 (a_a = cell rows)
    float ext1;       // sqrt((G^-1)_11): axis-1 extent of d^T G d <= 1
    float inv_det23;  // 1 / (G22 G33 - G23^2)
    float ext2, ext3; // sqrt(G33 / det23), sqrt(G22 / det23): in-plane extents per unit radius
    float HK[9];      // H[a][c] / K_a: Cartesian offset of one grid step along axis a
    float c2;         // (support radius / sigma)^2
    float wpref;      // dV / (2 pi)^{3/2}: theta = wpref / sigma^3 exp(-d^T G d / (2 sigma^2))
};

// Scalars that live on the device between CG kernels.
struct CgScalars {
    double rz[2];             // r.z of the current direction, double-buffered by parity
    double chi_norm;          // ||P chi_eff||
    double chi_sum;           // sum chi_eff
    double dinv_sum;          // sum 1 / D
    double res;               // relative residual after the last update
    double alpha;             // step length of the current iteration
    double e_start;           // energy of a supplied starting point (constraint plane)
    int iters;
    int done;
    int err;                  // QEQ_ERRBIT_*
    int pad;
};

// Kinds of kernel launches that the per-stage timers can bracket with events.
enum ProfKind {
    PK_SPREAD_R2C = 0,   // spread + axis-3 real-to-complex FFT
    PK_ROWS_FWD,         // axis-2 forward FFT
    PK_COLS_GREEN,       // axis-1 forward FFT, Green's function, axis-1 inverse FFT
    PK_ROWS_INV,         // axis-2 inverse FFT
    PK_C2R,              // axis-3 complex-to-real FFT
    PK_INTERP,           // back-interpolation + real-space product (CG matvec)
    PK_CG_UPDATE,
    PK_CG_DIR,
    PK_FINAL,            // final matvec epilogue: energies and forces
    PK_COUNT
};

struct ProfRec {
    int kind;
    int it;              // CG iteration of the launch, -1 outside the loop
    hipEvent_t a, b;
};

struct DeviceAxes {
    FftAxis ax[3];
};

struct BatchState;   // workspace of the batched solver (batched.hip)

struct qeq_plan {
    qeq_params prm;
    int n_max = 0;
    int dev = 0;
    hipStream_t stream = nullptr;

    // grid-dependent state
    int K[3] = {0, 0, 0};
    DeviceAxes axes;
    float2* tw[3] = {nullptr, nullptr, nullptr};
    float* bmod[3] = {nullptr, nullptr, nullptr};   // |b_a(m)|^2 per axis
    float* grid_r = nullptr;                        // real grid K1 K2 K3
    float2* grid_c = nullptr;                       // half spectrum [m3][m1][m2]
    int* bin_count = nullptr;                       // K1 K2 + 1
    int* bin_start = nullptr;
    int* bin_fill = nullptr;
    size_t grid_bytes = 0;

    // cell-dependent cache
    double cell_cached[9] = {0};
    bool theta_valid = false;
    double c_eta = 0.0;
    double* theta_tab = nullptr;                    // (2p-1)^3 mesh kernel values
    // virial: strain derivatives of the self-correction (d C_eta / d eps and
    // the six tables d Theta / d eps_ab), valid for the same cell as theta_tab
    bool strain_valid = false;
    double dc_eta[6] = {0, 0, 0, 0, 0, 0};
    double* strain_tab = nullptr;                   // 6 x (2p-1)^3
    double* vir_part = nullptr;                     // partial sums of the virial kernels
    size_t vir_cap = 0;                             // doubles

    // per-atom (sorted order unless noted)
    int* perm = nullptr;
    int* key = nullptr;           // original order: grid bin key
    double* frac = nullptr;       // n x 3
    int* home = nullptr;          // n x 4 (h1, h2, h3, cell)
    float* wts = nullptr;         // n x 3 x MAXP
    float* dwts = nullptr;        // n x 3 x MAXP
    double* sig = nullptr;
    double* Jv = nullptr;
    double* chi = nullptr;        // chi_eff (sorted)
    double* chi_raw = nullptr;    // chi (sorted)
    double* dself = nullptr;      // Gaussian self term + mesh self-correction
    double* dinv = nullptr;       // Jacobi preconditioner 1 / D
    double* selfgrad = nullptr;   // n x 3: d(theta^T Theta theta)/du
    double* q = nullptr;
    double* r = nullptr;
    double* pvec = nullptr;
    double* y = nullptr;
    double* forces_s = nullptr;   // n x 3 (sorted)
    double* gtmp = nullptr;       // n: final gradient vector
    double* fdst = nullptr;       // where the final matvec writes sorted forces
    // adjoint (tape of the last solve is q, y = E q, forces_s, geometry, pairs)
    double* q_adj = nullptr;      // adjoint solution a (sorted)
    double* y_adj = nullptr;      // matvec output buffer of the adjoint CG
    double* chi_adj = nullptr;    // -g, the adjoint right-hand side (sorted)
    double* adj_scratch = nullptr;// n x 3 scratch for the adjoint's final matvec
    double* tq = nullptr;         // n x 3: sum_g dtheta_i/du phi_q(g)

    // real-space cell list and pair list
    int ncell_alloc = 0;
    int* cell_count = nullptr;
    int* cell_start = nullptr;
    int* cell_fill = nullptr;
    int* cell_atoms = nullptr;
    int* rowptr = nullptr;        // n + 1
    int* rowcnt = nullptr;
    int* lanecnt = nullptr;       // [n_max][64] pairs per lane of the count pass (the fill's slices)
    size_t nnz_cap = 0;
    int* col = nullptr;
    float* kval = nullptr;
    float4* pdr = nullptr;        // (dx, dy, dz, K'(r)/r)
    long long nnz = 0;

    int* scan_tmp = nullptr;      // chunk totals of the multi-block scan
    size_t scan_cap = 0;

    // reductions
    double* part = nullptr;       // [2][nblk_max][QEQ_NPART]
    int nblk_max = 0;
    CgScalars* sc = nullptr;
    CgScalars* sc_host = nullptr; // pinned
    double* out_host = nullptr;   // pinned, 16 doubles
    int* nnz_host = nullptr;      // pinned: pair count of the last set-up
    CgScalars* sc_ring = nullptr; // pinned, 2: scalars of the CG chunks in flight
    hipEvent_t ring_ev[2] = {nullptr, nullptr};
    double* final_dev = nullptr;  // 16 doubles on device

    KParams kp;
    bool tape_valid = false;
    bool warm_rejected = false;   // the last solve discarded its q0

    BatchState* batch = nullptr;

    // spectral (small-k Woodbury) preconditioner; spc_kc <= 0 keeps Jacobi
    double spc_kc = 0.0;
    bool spc_active = false;      // built for the current geometry
    int spc_nm = 0;               // modes (half space)
    int spc_cap_m = 0;            // allocated modes
    int spc_cap_n = 0;            // allocated atoms
    int4* spc_modes = nullptr;    // integer triplets m, k = 2 pi H^-1 m
    float* spc_k2 = nullptr;      // |k|^2
    float* spc_winv = nullptr;    // 1 / w_k
    float* spc_wk = nullptr;      // w_k
    int spc_ncp = 0;              // table rows (2 nm padded to the tile)
    int spc_npad = 0;             // table columns (atoms padded)
    int spc_fsplit = 0;           // atom splits of t = Psi^T u
    float4* spc_atom = nullptr;   // (s1, s2, s3, sigma^2) per atom, sorted
    double* spc_dpinv = nullptr;  // 1 / D' per atom
    float* spc_sd = nullptr;      // D'^-1/2 per atom
    float* spc_u = nullptr;       // D'^-1/2 r per atom (padded)
    unsigned short* spc_psi = nullptr;   // bf16 table Psi, spc_ncp rows of spc_npad atoms
    double* spc_mats = nullptr;   // 6 dense (2m)^2 matrices: G, E, E2, P, Q, S
    float* spc_gpart = nullptr;   // split partial sums of Psi^T Psi
    double* spc_tpart = nullptr;  // split partial sums of Psi^T u
    double* spc_t = nullptr;      // Psi^T u
    double* spc_kpart = nullptr;  // k-split partial products of the dense series
    double* spc_s = nullptr;      // S t
    double* spc_wvec = nullptr;   // M^-1 r
    double* spc_m1 = nullptr;     // M^-1 1
    double* spc_ones = nullptr;   // all ones
    double* spc_scal = nullptr;   // [0] sum(M^-1 1), [1] ||E||_F^2, [2] min D'/D
    // non-periodic solve (direct pair sum); direct = the last solve's mode
    bool direct = false;
    bool np_valid = false;        // q and the pair-sum buffers of the last isolated solve
    bool geom_valid = false;      // sorted geometry and pair list of the last periodic set-up
    int np_cap = 0;               // atoms allocated
    int np_nsplit = 0;            // atom splits of the pair sum
    int np_tps = 0;               // tiles of 256 atoms per split
    double* np_pos = nullptr;     // double4 (x, y, z, sigma^2) per atom
    double* np_ypart = nullptr;   // [split][atom] partial products
    double* np_fpart = nullptr;   // [split][atom][3] partial force sums
    double* elem_buf = nullptr;   // 2 n_max: element source and product (caller order)

    // reciprocal part by direct Ewald sums instead of the mesh (qeq_use_ewald)
    bool ewald = false;           // requested for later periodic solves
    bool ew_active = false;       // the current solve's operator uses it
    int ew_nm = 0, ew_fs = 1, ew_fper = 0, ew_ms = 1, ew_mper = 0;   // modes, atom / mode splits
    int ew_cap_m = 0, ew_cap_n = 0;
    void* ew_modes = nullptr;     // int4 (m1, m2, m3, 0) per mode
    double* ew_w = nullptr;       // weights 2 (4 pi / V) exp(-eta^2 k^2 / 2) / k^2
    double* ew_sf = nullptr;      // [atom split][mode][2] structure-factor partials
    double* ew_y = nullptr;       // [mode split][atom] potential partials
    double* ew_f = nullptr;       // [mode split][atom][3] force partials
    double* ew_yrec = nullptr;    // reciprocal product, sorted order
    double* ew_frec = nullptr;    // reciprocal forces of the final product
    // SQNM instead of CG for qeq_solve (qeq_use_sqnm)
    bool sqnm = false;
    int sq_m = 10;                // history length
    int sq_cap_n = 0, sq_cap_m = 0;
    double* sq_S = nullptr;       // [m + 1][n_max] displacement ring
    double* sq_Y = nullptr;       // [m + 1][n_max] gradient-difference ring
    double* sq_g = nullptr;       // [2][n_max] gradients (current, trial)
    double* sq_part = nullptr;    // [blocks][SQ_NS_MAX] partial sums
    double* sq_sums = nullptr;    // [SQ_NS_MAX] reduced sums
    int* sq_desc = nullptr;       // [SQ_NS_MAX] sum descriptors (kind, i, j packed)
    double* sq_host = nullptr;    // pinned host copy of the sums
    int sq_iters = 0;             // iterations of the last SQNM solve (accepted + rejected)
    int sq_rejected = 0;          // steps undone after an energy rise

    // Gaussian-on-grid (plane-wave) operator instead of the split (qeq_use_planewave)
    bool planewave = false;       // requested for later periodic solves
    bool pw_active = false;       // the current solve's operator uses it
    double pw_support = 6.0;      // support radius in units of sigma_i
    PwGeom pw_geom{};
    int pw_cap_n = 0, pw_cap_k = 0;
    float* pw_ones = nullptr;     // unit moduli for the Green's function pass
    double* pw_y = nullptr;       // operator product, sorted order
    double* pw_f = nullptr;       // forces of the final product, sorted order
    double* pw_smax = nullptr;    // per-block maxima of sigma (host read once per set-up)
    bool fused_inverse = true;    // fused inverse axis-2 + complex-to-real slab pass where it fits
    bool fused_forward = true;    // fused spread + axis-3 + axis-2 forward plane pass where it fits
    bool fused_interp = true;     // CG products: complex-to-real pass fused with the interpolation
    int tile_set[3] = {0, 0, 0};  // qeq_set_tiles: spread rows, tile rows, axis-2 rows (0 = rule)
    float* mpart = nullptr;       // [2 MAXP][n_max] interpolation partials of the fused pass

    // the CG loop is replayed as a HIP graph of one chunk of iterations,
    // captured on a private stream and re-captured when its arguments change
    bool use_graphs = true;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<unsigned char> graph_key;

    // per-stage timers
    unsigned prof_mask = 0;
    int cur_it = -1;
    std::vector<ProfRec> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    double prof_ms[PK_COUNT] = {0};
    long long prof_n[PK_COUNT] = {0};
};

// Times one launch (or a sequence) when its kind is enabled: the start event
// goes to the first launch and the stop event to the last one of the scope,
// both recorded by the dispatches themselves (hipExtLaunchKernelGGL), so the
// interval is the kernels' own execution time.  Null events when disabled.
struct ProfScope {
    qeq_plan* pl;
    ProfRec rec;
    bool on;
    ProfScope(qeq_plan* p, int kind);
    ~ProfScope();
    hipEvent_t start() const { return on ? rec.a : nullptr; }
    hipEvent_t stop() const { return on ? rec.b : nullptr; }
};
void prof_flush(qeq_plan* pl, int live_iters);

// ------------------------------------------------------------------ helpers
int qeq_check(hipError_t e);
// With QEQ_POISON_ALLOC set in the environment, fresh floating-point device
// buffers are filled with NaN bytes: a result that reads memory no kernel
// wrote then turns into NaN instead of depending on what the allocator
// handed back (a check for the tests; off by default).
void debug_poison(void* p, size_t bytes);
template <typename T>
constexpr bool poisonable = std::is_floating_point<T>::value || std::is_same<T, float2>::value ||
                            std::is_same<T, float4>::value || std::is_same<T, double2>::value;
#define QEQ_TRY(x)                                   \
    do {                                             \
        int _rc = (x);                               \
        if (_rc != QEQ_OK) return _rc;               \
    } while (0)
#define QEQ_HIP(x) QEQ_TRY(qeq_check(x))

inline int nblocks(int n, int b = QEQ_BLOCK) { return (n + b - 1) / b; }
// blocks of the wave-per-atom interpolation kernel: QEQ_BLOCK / 64 atoms per
// block and round (waves stride over the atoms).  Up to 8 rounds per wave
// and at least 1024 blocks: fewer blocks mean fewer partial sums for every
// block of the next kernel to reduce (32,768 atoms: 1024 blocks, the CG
// update 8.5 -> 4.8 us for +1.6 us of interpolation).
inline int interp_blocks(int n) {
    const int b = (n + QEQ_BLOCK / 64 - 1) / (QEQ_BLOCK / 64);
    const int cap = b / 8 > 1024 ? (b + 7) / 8 : 1024;
    return b < cap ? b : cap;
}

// ------------------------------------------------------------------ setup kernels (setup.hip)
int launch_setup_clear(qeq_plan* pl);   // zeroes the CG scalars and the bin / cell counters
int launch_stage(qeq_plan* pl, const double* pos, const double* sigma, const double* J,
                 const double* chi);
int launch_sort_bins(qeq_plan* pl);
int launch_gather(qeq_plan* pl, const double* pos, const double* sigma, const double* J,
                  const double* chi);
// cell list, pair count and pair fill; the count goes to pl->nnz_host
// (pinned) without a synchronisation: after reading it the caller must call
// grow_pairs + launch_pair_fill again if it exceeds the capacity the fill saw
int launch_cells_and_pairs(qeq_plan* pl);
int launch_pair_fill(qeq_plan* pl);
int grow_pairs(qeq_plan* pl, size_t cap);
int launch_theta(qeq_plan* pl);          // mesh kernel table for the self-correction
int launch_selfcorr(qeq_plan* pl);
// the six d Theta / d eps_ab tables (6 x (2p-1)^3) for the virial
int launch_theta_strain(qeq_plan* pl, double* tabs);
// per block [sum q^2 theta^T dTheta_ab theta (6; 0 if tabs is null), sum q^2,
// sum q sigma^2]; nblocks(n) blocks of QEQ_NPART
int launch_self_strain(qeq_plan* pl, const double* tabs, double* part);
// d C_eta / d eps_ab (host, order 00, 11, 22, 01, 02, 12)
void reciprocal_self_strain(const double* H, const double* Hinv, double vol, double eta, double dC[6]);
// qeq_virial
int virial_impl(qeq_plan* pl, double* virial);
// spectral preconditioner (spectral.hip)
int spc_setup(qeq_plan* pl);                          // after the geometry set-up
// spc_wvec = M^-1 r, partials; u_ready: k_cg_update has written spc_u from r
int spc_apply(qeq_plan* pl, const double* r, const int* done, bool u_ready = false);
int spc_direction(qeq_plan* pl, int parity, int init);            // p from spc_wvec
void spc_free(qeq_plan* pl);
// non-periodic solve (direct.hip)
int np_setup(qeq_plan* pl, int n, const double* pos, const double* sigma, const double* J, const double* chi,
             double q_tot);
int launch_np_matvec(qeq_plan* pl, const double* src, double* dst, int mode);   // QEQ_MODE_CG / FINAL
void np_free(qeq_plan* pl);
int launch_final_tail(qeq_plan* pl, double* q_out, double* energies, double* forces_out);
// direct Ewald reciprocal part (ewald.hip)
int ew_setup(qeq_plan* pl);
int launch_ew_rec(qeq_plan* pl, const double* src, const int* done, bool fin);
int launch_ew_forces_add(qeq_plan* pl);
void ew_free(qeq_plan* pl);
// final product and host copies after a solve (api.hip); E src with the
// solve's operator, sorted order (api.hip)
int final_pass(qeq_plan* pl, double* q_out, double* energies, double* forces_out);
int operator_product(qeq_plan* pl, const double* src, double* dst);
// stabilised quasi-Newton minimisation instead of CG (sqnm.hip)
int sqnm_run(qeq_plan* pl, const double* q0, double* q_out, double* energies, double* forces_out, bool* conv);
void sqnm_free(qeq_plan* pl);
// Gaussian-on-grid operator (planewave.hip)
int pw_setup(qeq_plan* pl);
int launch_pw_rec(qeq_plan* pl, const double* src, const int* done, bool fin);
int launch_pw_forces_add(qeq_plan* pl);
void pw_free(qeq_plan* pl);
// element-resolved potentials (embed.hip)
int element_potentials_impl(qeq_plan* pl, const int32_t* species, int n_elem, double* out);
int launch_scan(qeq_plan* pl, const int* in, int* out, int m);
int launch_rhs_norm(qeq_plan* pl, const double* b);

// ------------------------------------------------------------------ mesh kernels (mesh.hip)
// Reciprocal potential of the charges src (sorted, FP64): real grid phi in grid_r.
int launch_mesh_potential(qeq_plan* pl, const double* src, const int* done);
// The CG product's mesh part: as launch_mesh_potential, or, where the fused
// complex-to-real + interpolation pass applies, the per-atom interpolation
// partials in pl->mpart instead of the real grid (*partials = true).
int launch_mesh_cg(qeq_plan* pl, const double* src, const int* done, bool* partials);
// whether the spread pass has a compile-time kernel for this length and tile width
bool spread_tile_compiled(int K3, int tws, int p);
size_t qeq_mesh_max_smem(const KParams& k);
// Inverse transforms only (grid_c already holds a spectrum) -> grid_r.
int launch_mesh_inverse(qeq_plan* pl);
// Passes 2-5 (axis-2 FFT, axis-1 FFT + Green's function + inverse, inverse
// axes 2 and 3) on a half spectrum that another pass 1 wrote into grid_c.
int launch_mesh_from_spectrum(qeq_plan* pl, const int* done);
// One launch of a single mesh pass (PK_SPREAD_R2C from src, or PK_C2R).
int launch_mesh_stage(qeq_plan* pl, int kind, const double* src);
int launch_write_green(qeq_plan* pl);
// G(m) d ln G / d eps_ab (component comp of 00, 11, 22, 01, 02, 12) into grid_c.
int launch_write_green_strain(qeq_plan* pl, int comp);
// Mesh virial partials of the charges src: spread, forward transforms and per
// block [sum e, sum e c k_a k_b]; mesh_virial_blocks() blocks of QEQ_NPART.
int launch_mesh_virial(qeq_plan* pl, const double* src, double* part);
int mesh_virial_blocks(const KParams& k);

// ------------------------------------------------------------------ solver kernels (solve.hip)
int launch_interp(qeq_plan* pl, const double* src, double* dst, int mode, int parity,
                  const float* mpart = nullptr);
int launch_cg_init_q(qeq_plan* pl, const double* q0);
int launch_cg_init_r(qeq_plan* pl);
int launch_start_energy(qeq_plan* pl);
int launch_cg_update(qeq_plan* pl, int parity);
int launch_cg_dir(qeq_plan* pl, int parity, int init);
int launch_final(qeq_plan* pl, double* q_out, double* energies, double* forces_out);
int launch_matvec_io(qeq_plan* pl, const double* v_orig, double* y_orig, int stage);

// ------------------------------------------------------------------ adjoint kernels (adjoint.hip)
int launch_adj_rhs(qeq_plan* pl, const double* dL_dq, double dL_dEelec);

// ------------------------------------------------------------------ batched solver (batched.hip)
void batch_free(qeq_plan* pl);

// ------------------------------------------------------------------ warm start (mlp.hip)
int launch_descriptors(qeq_plan* pl, const double* weights, int nf, const double* centers, double width, double rc,
                       float* G);
int launch_adj_gradients(qeq_plan* pl, double dL_dEqeq, double dL_dEelec, double* dL_dchi,
                         double* dL_dJ, double* dL_dpos);
