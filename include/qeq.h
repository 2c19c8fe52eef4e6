/*
 * qeq.h -- C ABI of the MI355X particle-mesh charge-equilibration library.
 *
 * Problem (RuNNer 2.0 paper, "Electrostatics and Charge Equilibration":
 * eq. elec_energy, eq. qeq_energy, eq. 4G_qeq_prime; SI "Fourth-Generation
 * HDNNPs and Charge Equilibration", eq. qeq).  Given positions r_i in a
 * periodic cell, Gaussian widths sigma_i, hardnesses J_i > 0,
 * electronegativities chi_i and a total charge Q_tot, find the charges q that
 * minimise
 *
 *     E_QEq(q) = E_elec(q) + sum_i (chi_i q_i + J_i q_i^2 / 2)   s.t.  sum_i q_i = Q_tot,
 *
 * where E_elec = q^T E q / 2 is the Coulomb energy of normalised Gaussian
 * charges (non-periodic kernel E_ii = 1/(sigma_i sqrt(pi)),
 * E_ij = erf(r_ij / (sqrt2 gamma_ij)) / r_ij, gamma_ij^2 = sigma_i^2 + sigma_j^2),
 * made periodic with a neutralising background and tin-foil boundary.
 * Stationarity gives (E + diag J) q = -chi + mu 1 (the SI's form; mu = -lambda
 * of the main text's bordered system).
 *
 * Method (paper, "Electrostatics Solvers", eq. matvec; SI "Particle--Particle--
 * Particle--Mesh Method"): conjugate gradients on the constraint plane, whose
 * matrix-vector product (E v)_i = dE_elec/dq_i is evaluated without forming E:
 * smooth particle-mesh Ewald with order-p cardinal B-splines, a 3-D FFT,
 * multiplication by the Gaussian-screened reciprocal kernel
 * 4 pi exp(-eta^2 k^2 / 2) / (V k^2), back-interpolation, plus a real-space
 * pair term [erf(r/(sqrt2 gamma)) - erf(r/(sqrt2 eta))]/r inside r_cut, the
 * Gaussian self term and the background term.
 *
 * Conventions for every call:
 *   - Atomic units (bohr, Hartree, e).
 *   - A cell is 9 doubles, row-major, ROWS = lattice vectors; it is a HOST
 *     pointer.  Every per-atom array is a DEVICE pointer on the plan's device,
 *     contiguous, owned by the caller.  pos is n x 3 row-major.
 *   - All device work is enqueued on the stream given to qeq_plan_create; the
 *     calls return after the stream has drained (they read back a status).
 *   - Return value: 0 on success; QEQ_NOT_CONVERGED (+1) when max_iter was
 *     reached (outputs hold the last iterate, stats are valid); a negative
 *     code on error (outputs untouched or partially written; no exception
 *     crosses the ABI).  qeq_strerror() names every code.
 *   - A plan is not thread-safe: one host thread at a time, and calls on one
 *     plan must not overlap.
 */
#ifndef QEQ_H
#define QEQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QEQ_OK             0
#define QEQ_NOT_CONVERGED  1
#define QEQ_EINVAL        -1  /* n < 1, J_i <= 0, sigma_i <= 0, non-finite input, singular cell */
#define QEQ_ECELL         -2  /* cell too skewed / grid too small for the spline order */
#define QEQ_ENOMEM        -3  /* device allocation failed */
#define QEQ_EHIP          -4  /* a HIP runtime call failed */
#define QEQ_EPLAN         -5  /* unsupported grid size or spline order, n > n_atoms_max */

typedef struct qeq_plan qeq_plan;   /* opaque; owns device workspace and the saved tape */

typedef struct qeq_params {
    double  eta;             /* std. dev. of the Ewald screening Gaussian (bohr); reciprocal
                                kernel exp(-eta^2 k^2 / 2), real-space erf(r/(sqrt2 eta))/r */
    double  r_cut;           /* real-space cutoff (bohr); all periodic images are included */
    double  max_spacing;     /* grid spacing bound (bohr), used when grid[0] == 0 */
    int32_t grid[3];         /* FFT grid K1,K2,K3: multiples of 4 with prime factors in
                                {2,3,5}, 12 <= K <= 512; grid[0] == 0 derives it per cell */
    int32_t spline_order;    /* p: even, 4 <= p <= 8 (cardinal B-spline M_p) */
    double  tol;             /* stop when ||P(A q + chi_eff)|| <= tol ||P chi_eff||, P = I - 11^T/N */
    int32_t max_iter;        /* CG iteration cap */
    int32_t self_correction; /* 1: replace each atom's mesh self-interaction by the exact
                                reciprocal self term (energy and force), 0: plain SPME */
    int32_t precond;         /* preconditioner of the projected CG: 0 Jacobi
                                (D_i = J_i + 1/(sigma_i sqrt(pi))), 1 spectral (the
                                long-wavelength Coulomb modes up to spectral_kcut on top of
                                Jacobi; see qeq_use_spectral_preconditioner) */
    double  spectral_kcut;   /* bohr^-1, used when precond == 1; <= 0 selects 0.2 */
} qeq_params;

typedef struct qeq_stats {   /* host memory */
    int32_t status;          /* same code the call returned */
    int32_t iters;           /* CG iterations taken */
    double  rel_resid;       /* recursive projected residual at exit (relative) */
    double  true_rel_resid;  /* projected residual of A q + chi recomputed at exit (relative) */
    double  mu;              /* Lagrange multiplier: (E + diag J) q + chi = mu 1 */
    double  e_qeq;           /* E_QEq at q */
    double  e_elec;          /* E_elec at q */
    int32_t q0_rejected;     /* 1 if the supplied q0 was worse than the cold start and replaced */
    int32_t reserved;
} qeq_stats;

/* Default parameters: eta 2.0, r_cut 11.0, max_spacing 0.8, grid derived,
   p = 6, tol 1e-6, max_iter 1000, self_correction 1, precond 0 (Jacobi),
   spectral_kcut 0.2. */
void qeq_params_default(qeq_params* p);

/* Create a plan for up to n_atoms_max atoms on the current HIP device.
   hip_stream: a hipStream_t (NULL = the default stream).  Returns QEQ_EPLAN
   for an unsupported grid or spline order, QEQ_EINVAL for bad parameters
   (including precond outside {0, 1} or a NaN spectral_kcut).  precond == 1
   has the effect of qeq_use_spectral_preconditioner(plan, spectral_kcut). */
int qeq_plan_create(qeq_plan** out, const qeq_params* params, int32_t n_atoms_max,
                    void* hip_stream);
int qeq_plan_destroy(qeq_plan* plan);

/* Solve the QEq problem (eq. 4G_qeq_prime) for one periodic structure.
   pos (n*3), sigma, J, chi (n each): device, read-only.
   q0 (n, device) or NULL: initial guess, projected onto sum = q_tot; NULL
   starts from q_tot/n.  A guess that starts farther from the solution than
   the cold start is discarded in favour of q_tot/n (stats->q0_rejected):
   for q_tot = 0 in the energy norm CG minimises (E_QEq(q0) >= E_QEq(0)),
   for charged cells by the projected residual (> ||P chi_eff||).
   q (n, device, out): charges.
   energies (2, device, out) or NULL: [E_QEq, E_elec].
   forces (n*3, device, out) or NULL: -dE_QEq/dr at the solution.  At the
   stationary point this equals -dE_elec/dr at fixed q, so no extra solve is
   needed (SI eq. 4g_force_trick with a constant chi and J).
   stats (host, out) or NULL.
   The call saves a tape (sorted geometry, pair list, q, potential) that
   qeq_backward uses; the next solve on the plan replaces it. */
int qeq_solve(qeq_plan* plan, int32_t n, const double* pos, const double* cell,
              const double* sigma, const double* J, const double* chi, double q_tot,
              const double* q0, double* q, double* energies, double* forces,
              qeq_stats* stats);

/* Solve the QEq problem (eq. 4G_qeq_prime) for one isolated (non-periodic)
   system: a molecule or cluster in any total-charge state (the paper's
   motivation for 4G potentials of non-periodic systems).  The Coulomb
   operator is the paper's kernel between normalised Gaussians with no
   images, E_ii = 1/(sigma_i sqrt(pi)), E_ij = erf(r_ij/(sqrt2 gamma_ij))/r_ij
   (Electrostatics and Charge Equilibration section), summed directly over
   all pairs: O(n^2) work per CG product, no grid, no cutoff, no background.
   Arguments, ownership, q0 handling, outputs and errors as qeq_solve; there
   is no cell and the plan's grid, eta and r_cut are unused (tol and
   max_iter apply).  Positions may lie anywhere (coincident atoms are
   allowed: the kernel takes its r -> 0 limit).  The call leaves no tape:
   qeq_backward and qeq_virial return QEQ_EINVAL until the next periodic
   solve. */
int qeq_solve_nonperiodic(qeq_plan* plan, int32_t n, const double* pos, const double* sigma,
                          const double* J, const double* chi, double q_tot, const double* q0,
                          double* q, double* energies, double* forces, qeq_stats* stats);

/* Element-resolved electrostatic potentials of the last solve on this plan:
   the embedding features of the paper's ee4G variant (Electrostatics and
   Charge Equilibration section: element-specific potentials at each atomic
   site from the equilibrated charges, appended to the feature vector).
     gamma[i * n_elem + z] = sum_j E_ij q_j [species_j = z]
                             - [species_i = z] q_i / (sigma_i sqrt(pi)),
   i.e. the potential at atom i of the charges of element z without the
   atom's own Gaussian self term; E is the Coulomb operator of that solve
   (qeq_solve: periodic images, mesh, pairs, self and background terms;
   qeq_solve_nonperiodic: the direct pair sum).  Summed over z and completed
   with q_i/(sigma_i sqrt(pi)) + J_i q_i + chi_eff,i it gives the Lagrange
   multiplier mu at every atom (the stationarity of the solve).
   species (n, int32, device, caller order): element index of each atom;
   atoms outside [0, n_elem) belong to no channel.  n_elem in [1, 16].
   gamma (n * n_elem, FP64, device, caller order, out).
   Cost: n_elem operator products.  The tape for qeq_backward / qeq_virial is
   kept.  QEQ_EINVAL without a preceding successful solve (or after
   qeq_matvec / qeq_solve_batched, which replace it) or for bad arguments. */
int qeq_element_potentials(qeq_plan* plan, const int32_t* species, int32_t n_elem, double* gamma);

/* Gradient of a loss L(q, E_QEq, E_elec) through the last solve on this plan
   (SI eq. 4g_force_trick: Lagrange / adjoint route, one extra linear solve
   with the same operator instead of 3N charge derivatives).
   dL_dq (n, device, caller order) or NULL for zero; dL_dEelec, dL_dEqeq:
   scalar weights of the two energies, in that order (E_elec first).
   Outputs (device, caller order, each may be NULL):
     dL_dchi (n) = -a + dL_dEqeq q,
     dL_dJ   (n) = -a q + dL_dEqeq q^2 / 2,
     dL_dpos (n*3) = (dL_dEqeq + dL_dEelec) dE_elec/dr|_q - d(a^T E q)/dr,
   where [E + diag J, 1; 1^T, 0][a; nu] = [dL_dq + dL_dEelec E q; 0].
   stats (host) report the adjoint CG.  Needs a preceding successful
   qeq_solve on the same plan (QEQ_EINVAL otherwise); gradients with respect to
   sigma and the cell are not provided. */
int qeq_backward(qeq_plan* plan, const double* dL_dq, double dL_dEelec, double dL_dEqeq,
                 double* dL_dchi, double* dL_dJ, double* dL_dpos, qeq_stats* stats);

/* Virial of the last solve on this plan (SI "Stress Tensor": the stress is
   sigma = (1/V) dE/d eps and the virial an MD code takes is -V sigma):
     virial (9 doubles, device, out, row-major) W_ab = -dE/d eps_ab
   for the homogeneous strain r -> (1 + eps) r of positions and lattice
   vectors (fractional coordinates fixed); symmetric.  E is the plan's
   discretised E_elec at the solution charges: mesh energy, real-space pairs,
   mesh self-correction, background (charged cells).  At the QEq solution
   this also equals -dE_QEq/d eps with the charges re-equilibrated, since
   E_QEq is stationary on sum(q) = Q and J, chi do not depend on the
   geometry.  The stress is -W / V with V = |det cell|.
   Needs a preceding successful qeq_solve on the plan (QEQ_EINVAL otherwise,
   also after qeq_matvec or qeq_descriptors, which replace the geometry).
   Runs one charge spread and two forward transform passes, the pair list and
   per-atom terms; the first call for a cell also builds six strain tables of
   the mesh self-correction (six inverse mesh transforms).  Synchronises the
   plan's stream. */
int qeq_virial(qeq_plan* plan, double* virial);

/* y = E v with the plan's particle-mesh operator (no J), for checking the
   matrix-vector product of eq. matvec on its own.  parts is a bit mask:
   1 reciprocal (mesh) part, 2 real-space pair part, 4 self terms (Gaussian
   self energy and mesh self-correction), 8 background term; 15 = all of E.
   The mesh part takes the path of the CG products (see qeq_use_fused_interp).
   v, y: n doubles on the device. */
int qeq_matvec(qeq_plan* plan, int32_t n, const double* pos, const double* cell,
               const double* sigma, const double* v, double* y, int32_t parts);

/* ------------------------------------------------------------------------
   Batched solve: many independent structures in one persistent launch.
   ------------------------------------------------------------------------ */

#define QEQ_BATCH_NMAX 1024   /* largest structure of the batched path */

/* Solve eq. 4G_qeq_prime for n_struct independent periodic structures of
   uneven size (the paper treats structures independently and distributes them
   over ranks; here one launch with one workgroup per structure at a time, the
   order longest first).  Structure s owns atoms atom_offsets[s] ..
   atom_offsets[s+1]-1 of the concatenated arrays.
   atom_offsets (n_struct + 1, HOST, non-decreasing), cells (n_struct x 9,
   HOST, rows = lattice vectors), q_tot (n_struct, HOST).
   pos (3 per atom), sigma, J, chi (1 per atom): DEVICE, read-only.
   q0 (DEVICE, 1 per atom) or NULL: starting charges, treated per structure as
   in qeq_solve.  q (DEVICE, out), energies (DEVICE, n_struct x 2 =
   [E_QEq, E_elec], out, or NULL), forces (DEVICE, 3 per atom, out, or NULL),
   stats (HOST, n_struct, out, or NULL).
   Each structure gets its own grid from the plan's max_spacing (or the plan's
   fixed grid), axis lengths up to 64, and at most QEQ_BATCH_NMAX atoms; the
   plan's eta, r_cut, spline order, tol, max_iter and self_correction apply to
   all.  Per-structure failures (invalid input or cell: QEQ_EINVAL; too many
   atoms, unsupported grid or r_cut above 4 perpendicular widths: QEQ_EPLAN)
   are reported in stats[s].status and do not stop the other structures; such
   structures leave q, energies and forces unwritten.  The return value is the
   most negative per-structure status, else QEQ_NOT_CONVERGED if any structure
   did not converge, else QEQ_OK.  Does not touch the tape of qeq_solve /
   qeq_backward other than invalidating it. */
int qeq_solve_batched(qeq_plan* plan, int32_t n_struct, const int32_t* atom_offsets,
                      const double* pos, const double* cells, const double* sigma,
                      const double* J, const double* chi, const double* q_tot,
                      const double* q0, double* q, double* energies, double* forces,
                      qeq_stats* stats);

/* Launch shape of qeq_solve_batched: threads per workgroup (1024; other
   sizes are QEQ_EINVAL) and workgroups per compute unit (1 .. 8; the launch
   has that many per CU, as many as fit run at once).  Does not change results beyond FP32 rounding
   order.  Defaults 1024, 1. */
int qeq_batched_config(qeq_plan* plan, int32_t threads, int32_t wg_per_cu);

/* Milliseconds of the batched kernels (HIP events) accumulated since the
   last reset; reset != 0 clears the counter. */
double qeq_batched_last_ms(qeq_plan* plan, int32_t reset);

/* Per-structure time breakdown of the last qeq_solve_batched call, measured
   inside the kernel with the GPU's constant 100 MHz clock by each structure's
   workgroup: us[s * 8 + k] = microseconds in phase k of structure s, k =
   0 staging / C_eta, 1 pair list, 2 Green table and mesh self-correction,
   3 spreading, 4 FFT passes, 5 interpolation and pair product, 6 CG vector
   updates and reductions, 7 total.  us: host, n_struct x 8 doubles.
   Returns 8, or QEQ_EINVAL if n_struct exceeds the last call's batch. */
int qeq_batched_phase_us(qeq_plan* plan, int32_t n_struct, double* us);

/* ------------------------------------------------------------------------
   Learned warm start (a small per-element network predicts initial charges).
   ------------------------------------------------------------------------ */

/* Radial descriptors (paper eq. g2 with the SI cosine cutoff, inner radius 0),
   optionally weighted per neighbour (the paper's weighted ACSFs, whose terms
   carry a scalar prefactor of the neighbour):
     G_i,mu = sum_{j, images, r_ij < r_cut} w_j exp(-(r_ij - c_mu)^2 / (2 width^2))
                                             (cos(pi r_ij / r_cut) + 1) / 2,
   mu < n_feat <= 32, over all neighbours (not element-resolved); w_j = 1 when
   weights is NULL.  Runs the plan's geometry set-up (which replaces the tape of
   the last solve), so r_cut must not exceed the plan's real-space cutoff.
   weights: device, n doubles, caller order, or NULL.  centers: host, n_feat
   doubles.  G: device, n x n_feat floats, caller order.
   pos == NULL reuses the geometry (sorted atoms, pair list) of the last
   qeq_solve or qeq_descriptors call on this plan with the same n, skipping
   the set-up and keeping the solve's tape; cell and sigma are then ignored
   (QEQ_EINVAL if there is no such geometry). */
int qeq_descriptors(qeq_plan* plan, int32_t n, const double* pos, const double* cell,
                    const double* sigma, const double* weights, int32_t n_feat,
                    const double* centers, double width, double r_cut, float* G);

/* Element networks 16-32-32-1, tanh hidden layers, linear output (SI
   feed-forward networks), one per element; inputs scaled per element as
   (G - mean) / (max - min) (SI feature scaling) and clipped to [-1.5, 1.5]
   (atoms that leave the training range do not saturate the network).  Products run on BF16 MFMA
   (operands rounded to nearest even) with FP32 accumulation; biases, tanh and
   the output layer in FP32.
   params: device floats, element e at offset 1664 e, packed as
     W1[32][16] | b1[32] | W2[32][32] | b2[32] | W3[32] | b3   (1633 used).
   stats: device floats [n_species][3][16] = mean, min, max per feature.
   species: device int32 in [0, n_species), n_species <= 4.
   All calls enqueue on `stream` (a hipStream_t) and do not synchronise.   */

/* Floats of scratch workspace that mlp_train_step / mlp_feature_stats need. */
int64_t mlp_workspace_floats(int32_t n_species);

/* Per-element mean / min / max of the 16 features over the given atoms. */
int mlp_feature_stats(const float* G, const int32_t* species, int32_t n, int32_t n_species,
                      float* stats, float* workspace, void* stream);

/* out[i] (device double) = network of species[i] applied to G[i]; pass out
   as the q0 of qeq_solve (the solve projects it onto sum = Q_tot, which is
   the paper's constraint projection of predicted charges). */
int mlp_forward(const float* G, const int32_t* species, int32_t n, int32_t n_species,
                const float* params, const float* stats, double* out, void* stream);

/* One training step on the batch: L = 1/2 mean (y - target)^2 (SI loss with
   the 1/2 prefactor), gradients by a hand-written backward pass (BF16 MFMA,
   FP32 accumulate), then Adam (beta1 0.9, beta2 0.999, eps 1e-8; SI) with
   learning rate lr at step `step` (>= 1; step 0 computes loss and gradients
   only).  loss (device, 1 float) and grad_out (device, like params) may be
   NULL.  workspace: device, at least mlp_workspace_floats floats. */
int mlp_train_step(const float* G, const int32_t* species, const double* target, int32_t n,
                   int32_t n_species, const float* stats, float* params, float* adam_m,
                   float* adam_v, int32_t step, float lr, float* workspace,
                   int64_t workspace_floats, float* loss, float* grad_out, void* stream);

/* mlp_train_step without the workspace argument, for callers that cannot
   allocate device memory (code under stream capture, serving loops,
   harnesses that forbid hipMalloc): the partial gradients and loss partials
   live in a fixed array of the library on each device (7.0 MB:
   mlp_workspace_floats(4) floats, enough for any n_species <= 4 and any n),
   looked up once per device on the first call.  Calls no hipMalloc / hipFree.
   Arguments, outputs and errors as mlp_train_step (QEQ_EINVAL for
   n_species > 4 or bad pointers); results equal mlp_train_step's up to the
   FP32 rounding order of the gradient sums.  Every call on one device shares
   that device's array: calls that overlap on one device (other streams,
   other host threads) race and must be serialised by the caller; nothing in
   the array needs to start at zero (each call overwrites what it reads). */
int mlp_train_step_noalloc(const float* G, const int32_t* species, const double* target, int32_t n,
                           int32_t n_species, const float* stats, float* params, float* adam_m,
                           float* adam_v, int32_t step, float lr, float* loss, float* grad_out,
                           void* stream);

/* The CG loop of qeq_solve / qeq_backward runs as a replayed HIP graph of
   12 iterations, 4 with the spectral preconditioner (captured on a private
   stream, launched on the plan's stream,
   re-captured when the geometry or buffers change); enable = 0 launches every
   kernel separately instead.  Results are the same either way up to the
   rounding order of the mesh atomics.  Default on.  While per-stage timers
   are enabled (qeq_profile) the loop launches kernels one by one. */
int qeq_use_graphs(qeq_plan* plan, int32_t enable);

/* Where a g1 slab of the half spectrum (K2 (K3/2 + 1) complex values) fits
   in the LDS of one compute unit (grids 96^3 and 192^3 with K1 >= 64), the
   inverse axis-2 transform and the axis-3 complex-to-real transform run as one
   pass (eq. matvec's back-transform without the intermediate grid round
   trip); enable = 0 runs them as two passes.  Both give the same potential
   up to FP32 rounding.  Default on. */
int qeq_use_fused_inverse(qeq_plan* plan, int32_t enable);

/* Where a g1 plane of the half spectrum fits in the LDS of one compute unit
   (192^3 grids with K1 >= 64, spline order 6), the charge spreading of eq.
   matvec, the axis-3 real-to-complex transform and the forward axis-2
   transform run as one pass, with one fixed-point scale per grid row; enable
   = 0 runs the spread pass (row tiles) and the axis-2 pass.  Both give the
   same spectrum up to FP32 rounding.  Default on. */
int qeq_use_fused_forward(qeq_plan* plan, int32_t enable);

/* The CG products of qeq_solve / qeq_backward: enable != 0 (default) runs the
   axis-3 complex-to-real transform of each (g1, row-tile) block and the
   back-interpolation of eq. matvec (sum_g theta_i(g) phi(g)) over that tile in
   one pass, so the real potential grid is neither written nor read again;
   each atom's 2p tile partials are summed in a fixed order with its
   real-space pair product.  enable = 0 writes the potential grid and
   interpolates from it (the path the final energies and forces always use).
   Both give the same product up to FP32 rounding order.  Applies where the
   axis-2 tile is at least p - 1 rows wide (every supported grid with p <= 8
   at 8- or 16-row tiles). */
int qeq_use_fused_interp(qeq_plan* plan, int32_t enable);

/* Tile widths of the mesh passes for later solves on this plan, replacing the
   built-in rule (spread tiles whose block fits 26 KB of LDS with at least two
   blocks per CU, axis-1 / complex-to-real tiles within 48 KB, fewer axis-2
   rows per block for grids beyond the Infinity Cache): spread_rows = axis-2 rows per
   block of the spread + axis-3 real-to-complex pass, tile_rows = axis-2 rows
   of the axis-1 and complex-to-real passes, fft_rows = rows per block of the
   axis-2 pass; 0 keeps the rule for that one.  Powers of two, 4..32 rows (1..32
   for fft_rows; spread_rows also 12 or 24), else QEQ_EINVAL.  A choice that
   does not divide the grid, is narrower than p - 1 rows or needs more than
   60 KB of LDS, or a spread width of 12 or 24 rows on a grid length without
   a compiled kernel for it, makes the next solve return QEQ_EPLAN.  The widths change the blocking only: results agree
   to FP32 rounding order.  paper_2607_17978_amd.autotune measures them. */
int qeq_set_tiles(qeq_plan* plan, int32_t spread_rows, int32_t tile_rows, int32_t fft_rows);

/* Reciprocal-space method of later qeq_solve calls on this plan: enable = 0
   (default) the particle mesh (B-spline spreading, FFT, Green's function,
   interpolation); enable != 0 direct Ewald summation (SI "Ewald Summation";
   the paper's O(N^3/2) solver for small cells): the explicit sum over the
   reciprocal vectors 0 < |k| <= k_max of the half space with
   exp(-eta^2 k^2 / 2) >= 1e-12, weights 2 (4 pi / V) exp(-eta^2 k^2 / 2) / k^2,
   through structure factors, O(n M) per CG product for M such vectors
   (M grows with the cell volume: about 2,800 at 64 atoms in an 18.6-bohr
   cube with eta = 2, 22,000 at 512 atoms of the same density).  The real-space
   pairs (plan r_cut), self and background terms, CG, energies and forces are
   unchanged; there is no mesh and no mesh self-correction (the sums are
   exact).  QEQ_EPLAN from qeq_solve when a cell needs more than 2^20
   vectors.  The adjoint, the virial and the element potentials use the
   mesh: after an Ewald solve qeq_backward, qeq_virial and
   qeq_element_potentials return QEQ_EINVAL.  The batched and non-periodic
   solves are not affected.  Enabling it switches qeq_use_planewave off. */
int qeq_use_ewald(qeq_plan* plan, int32_t enable);

/* Operator of later qeq_solve calls on this plan: enable != 0 the
   Gaussian-on-grid ("plane-wave") evaluation of the paper's eq. matvec
   ("Electrostatics Solvers": the Gaussian charge densities themselves are put
   on the grid, the potential comes from the Poisson kernel 4 pi / G^2 via
   FFT, and (A q)_i is the integral of that potential over atom i's density),
   with no Ewald split: no real-space pairs, no self or background terms, no
   spline moduli, no screening.  Atom i's density is sampled out to
   support * sigma_i (support = 0 selects 6; accepted 3 .. 12, else
   QEQ_EINVAL): about 4 (pi/3) (support sigma_i)^3 / dV grid points per atom
   instead of p^3 for the spline spread.  The grid is the plan's (grid or
   max_spacing); sigma_i well above the spacing keeps the aliasing error small
   (about 1e-8 relative in the operator at 0.8 bohr and sigma >= 1).
   enable = 0 (default) restores the split particle mesh.  The charges,
   energies, mu and forces are those of the same CG; the final pass adds the
   forces -q_i / sigma_i^2 sum_g theta_i(g) phi(g) (r_g - r_i).  QEQ_EPLAN
   from qeq_solve when the widest atom's support exceeds four grid lengths
   along an axis.  After such a solve qeq_backward, qeq_virial and
   qeq_element_potentials return QEQ_EINVAL.  Enabling it switches
   qeq_use_ewald off; the batched and non-periodic solves are not affected.
   The spread adds FP32 values with atomics, so repeated solves agree to FP32
   rounding, not bit for bit. */
int qeq_use_planewave(qeq_plan* plan, int32_t enable, double support);

/* Solver of later qeq_solve calls on this plan: enable != 0 stabilised
   quasi-Newton minimisation (SQNM; the paper's alternative to conjugate
   gradients in its solver comparison) of E_QEq on the plane
   sum(q) = Q_tot instead of projected CG; enable = 0 (default) CG.  The
   minimiser works in the Jacobi metric (D_i = J_i + 1/(sigma_i sqrt(pi))),
   keeps the last `history` displacement / gradient-difference pairs
   (0 selects 10; 1 .. 16 accepted, else QEQ_EINVAL), builds the Hessian in
   their well-conditioned span (overlap eigenvalues above 1e-4 of the
   largest), takes quasi-Newton steps there and scaled steepest-descent steps
   in the complement, undoes a step that raises the energy (halving the
   step scale and clearing the history; energy changes below 1e-6 of the
   energy's terms count as rounding) and stops at the relative residual
   max(tol, 1e-7): its gradient is the FP32 operator's, whose residual floor
   is near 1e-7 (the CG path's true-residual check allows 2 max(tol, 1e-7)
   for the same reason).  One host synchronisation per iteration (the m x m
   eigenproblems run on the host); no graph replay.  The charges, energies,
   forces, mu and true residual come from the same final pass as after CG;
   stats->iters counts SQNM iterations, undone ones included.  Works with
   the mesh, Ewald and Gaussian-on-grid operators; the spectral
   preconditioner is not used by it; the tape for qeq_backward / qeq_virial
   / qeq_element_potentials is kept (the adjoint solve itself stays CG).
   qeq_solve_nonperiodic and qeq_solve_batched keep CG. */
int qeq_use_sqnm(qeq_plan* plan, int32_t enable, int32_t history);

/* Preconditioner of the projected CG in qeq_solve / qeq_backward.
   k_cut <= 0 (default): Jacobi, D_i = J_i + 1/(sigma_i sqrt(pi)).
   k_cut > 0 (bohr^-1): spectral preconditioner for the long-wavelength
   Coulomb modes whose eigenvalues make the iteration count grow with N
   (the Electrostatics Solvers section's observation).  The exact plane-wave
   Coulomb part at the reciprocal vectors 0 < |k| <= k_cut (at most the 384
   nearest, half space) is added to the Jacobi diagonal as a low-rank term,
     M = D' + Phi W Phi^T,  W = diag(2 (4 pi / V) / k^2),
     Phi = [F_i(k) cos(k.r_i) | F_i(k) sin(k.r_i)],  F_i(k) = exp(-sigma_i^2 k^2 / 2),
     D' = D - diag(Phi W Phi^T),
   and applied by the Woodbury identity with the small inverse built once per
   geometry.  The converged charges are the same as with Jacobi (the solve
   tolerance applies unchanged); k_cut ~ 0.2 bohr^-1 cuts the cold-start
   iterations of a 32,768-atom cell from 57 to 17.  If the geometry
   falls outside the range where the construction is safe (D' <= 0.1 D or a
   weakly dominant small matrix) the solve uses Jacobi.  QEQ_EINVAL for NaN. */
int qeq_use_spectral_preconditioner(qeq_plan* plan, double k_cut);

/* Per-stage timers (the paper's per-stage timing of a step, here with HIP
   events on the plan's stream).  kind_mask selects which launch kinds are
   bracketed with events during later calls; 0 switches timing off.  Kinds:
     0 spread + axis-3 R2C FFT      1 axis-2 forward FFT
     2 axis-1 FFT + Green + inverse 3 axis-2 inverse FFT
     4 axis-3 C2R FFT               5 interpolation + pair product (CG)
     6 CG update                    7 CG direction
     8 final energies / forces
   CG-loop launches that found the solve already converged are not counted. */
int qeq_profile(qeq_plan* plan, uint32_t kind_mask);

/* Copies accumulated milliseconds and launch counts for the first n_kinds
   kinds into total_ms / launches (host arrays, may be NULL), optionally
   resets them, and returns the number of kinds the library knows (9).
   Synchronises the plan's stream. */
int qeq_profile_read(qeq_plan* plan, double* total_ms, int64_t* launches, int32_t n_kinds,
                     int32_t reset);

/* Average duration (microseconds, *avg_us) of one launch of a single mesh
   pass, timed with HIP events around `reps` back-to-back launches on the
   plan's stream with the geometry and charges of the last successful solve:
   kind 0 = spread + axis-3 R2C FFT (from the solve's q), kind 4 = axis-3 C2R
   FFT (the other passes work in place and are not offered).  The passes only
   overwrite the plan's mesh buffers; the tape for qeq_backward stays valid.
   kind 9 = one CG product of the direct pair sum (pair kernel + epilogue)
   on the charges of the last qeq_solve_nonperiodic call.
   QEQ_EINVAL without a preceding solve of the matching kind or for another
   kind. */
int qeq_time_kernel(qeq_plan* plan, int32_t kind, int32_t reps, double* avg_us);

const char* qeq_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* QEQ_H */
