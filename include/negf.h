/*
 * negf.h -- C ABI of the MI355X (gfx950) NEGF hot-path library (libnegf.so).
 *
 * The library solves, at every energy point E (and transverse momentum, passed
 * as a separate device H(k)), the retarded and lesser/greater equations of
 * non-equilibrium Green's functions on block-tridiagonal operators:
 *
 *   Eq. (1)  G^R = (A - B^R)^{-1},   A - B^R = E S - H - Sigma^R_B - Sigma^R_sc
 *   Eq. (2)  (G^R)^{-1} G^<> (G^A)^{-1} = B^<>,  i.e.  G^<> = G^R Sigma^<> G^A
 *
 * where Sigma_B is the open-boundary term of the two leads (the paper adds it
 * to B without showing it, Section II after Eq. (3)) and Sigma_sc an optional
 * block-diagonal scattering self-energy.  Only the blocks inside the sparsity
 * pattern of A are returned (Section II, the paragraph after Fig. 3): the
 * diagonal and first off-diagonal blocks.  The selected inversion is the
 * recursive Green's function (RGF) algorithm the paper names as the
 * sequential solver; energies are independent (same paragraph) and are the
 * batch axis of every call.
 *
 * Conventions shared by all calls
 * -------------------------------
 *  - Complex data are interleaved (re, im) pairs of double (complex128),
 *    C-contiguous row-major b x b blocks: the memory layout of torch / NumPy
 *    complex128 arrays.  Block i of an [nb][b][b] array starts at i*b*b.
 *  - Unless stated otherwise, every array pointer is a DEVICE pointer owned by
 *    the caller, 16-byte aligned.  The library allocates no device memory in
 *    any call: scratch comes from the caller's workspace (negf_workspace_bytes).
 *  - Outputs must not overlap the inputs, each other or the workspace.  Until
 *    a call's work has finished their contents are intermediate (the G^<> upper
 *    blocks, for instance, hold a forward-sweep product until the backward
 *    sweep writes the result there).
 *  - A "point" is one (problem, energy) pair.  Points are numbered problem by
 *    problem in order, energies in order inside a problem.  Per-point outputs
 *    are stored point-major, each point's part sized by its own (nb, b):
 *    e.g. GR_diag holds, for each point, nb blocks of b x b.
 *  - The device sits at real energy; z = E + i*eta enters only the leads.
 *  - Leads repeat the first and last device cell: left lead cell (H_00, S_00)
 *    with coupling (H_01, S_01), right lead cell (H_{N-1,N-1}, S_{N-1,N-1})
 *    with coupling (H_{N-2,N-1}, S_{N-2,N-1}).  Their surface Green's functions
 *    come from Sancho-Rubio decimation in double precision.
 *  - Errors: argument errors (null required pointer, nb < 2, b < 1, b > 1024,
 *    workspace too small, misaligned pointer) return NEGF_EINVAL
 *    synchronously and enqueue nothing.  All work is enqueued on `stream`
 *    (a hipStream_t; NULL = the null stream).  Numerical outcomes are written
 *    per point into the device array info[] (LAPACK style): NEGF_OK,
 *    NEGF_ENOCONV (decimation not converged or residual above the accept
 *    threshold), NEGF_ESINGULAR (zero pivot), NEGF_ENONFINITE (NaN/Inf).
 *    A HIP launch failure returns NEGF_EHIP.
 *  - Synchronisation: none.  Every call only enqueues work on `stream` and
 *    reads nothing back; the decimation enqueues exactly sr_max_iter steps
 *    and masks each (point, lead) pair out of the later steps once it has
 *    converged, so calls may be captured into a graph (steps after the last
 *    pair has converged launch workgroups that exit at once).
 *  - Thread safety: calls on distinct workspaces and streams may run
 *    concurrently.  The profiling counters are process-global.
 */
#ifndef NEGF_H
#define NEGF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NEGF_OK = 0,
  NEGF_EINVAL = 1,
  NEGF_ENOCONV = 2,
  NEGF_ESINGULAR = 3,
  NEGF_ENONFINITE = 4,
  NEGF_EHIP = 5,
  NEGF_ENOMEM = 6
} negf_status;

/* Arithmetic of the dense block products of the RGF sweeps.  Inversions,
 * block sums, residuals and the lead decimation are double in every mode.
 *  PLAIN_FP64    : every product in double (the reference method)
 *  FP32_REFINE   : backward retarded products single (complex64 operands,
 *                  single accumulation), each block followed by one
 *                  double-precision residual correction of its three blocks
 *                  from the local identities of the backward step; everything
 *                  else double
 *  FP32_NOREFINE : every sweep product single, no correction (diagnostic)   */
typedef enum { NEGF_PLAIN_FP64 = 0, NEGF_FP32_REFINE = 1, NEGF_FP32_NOREFINE = 2 } negf_precision;

/* One block-tridiagonal device (Section II: BT shape imposed on A and B).
 * H_diag [nb][b][b] and H_upper [nb-1][b][b] (H_{i,i+1}) are required; the
 * lower blocks are H_{i+1,i} = H_{i,i+1}^H.  S_diag/S_upper == NULL means
 * S = I.  sig_r_sc / sig_l_sc / sig_g_sc: optional block-diagonal
 * scattering self-energies [nb][b][b] (retarded, lesser, greater), the same
 * for every energy unless the problem's sc_stride says otherwise; NULL =
 * none (ballistic). */
typedef struct negf_device {
  int32_t nb, b;
  const void* H_diag;
  const void* H_upper;
  const void* S_diag;
  const void* S_upper;
  const void* sig_r_sc;
  const void* sig_l_sc;
  const void* sig_g_sc;
} negf_device;

/* A device and its list of energies (device array of n_e doubles).
 * eta: lead broadening; mu_l, mu_r, kT: contact Fermi levels and temperature
 * for Sigma^<_B = i f Gamma, Sigma^>_B = -i (1 - f) Gamma.
 * sc_stride: 0, or the distance in complex elements (>= nb b b) between the
 * scattering self-energies of consecutive energies, so that energy e reads
 * sig_*_sc + e sc_stride: energy-dependent self-energies, as the
 * self-consistent loop of Fig. 1 produces them (Eq. (3)).  The point queue
 * (negf_plan_run_queue) takes only sc_stride = 0. */
typedef struct negf_problem {
  negf_device dev;
  int32_t n_e;
  const double* energies;
  double eta, mu_l, mu_r, kT;
  int64_t sc_stride;
} negf_problem;

/* Optional knobs (pass NULL for the defaults in brackets). */
typedef struct negf_options {
  double sr_tol;        /* decimation stops when ||a||_F, ||c||_F <= tol ||d||_F  [1e-14] */
  int32_t sr_max_iter;  /* decimation steps enqueued (iteration cap)             [64]    */
  double sr_accept;     /* normalised Dyson residual above which info=ENOCONV   [1e-8]  */
  int32_t batch;        /* points in flight per group (0: all points of the call) [0]   */
  int32_t inv_nb;       /* panel width of the block inversion (16 or 32)          [16]  */
  int32_t xcd_remap;    /* 1: place the tiles of one matrix on one XCD            [1]   */
  int32_t gemm_tile;    /* product tile: 1 = 64x64, 2 = 128x64, 3 = 128x128,
                           4 = 64x64 with 8 waves, 5 = 128x64 with 16 waves,
                           6 = 32x32; a launch whose 64x64 tiles would number
                           fewer than two per CU (a few points per call) runs
                           on 32x32 tiles whatever is set here                   [1]   */
  int32_t gemm_tile_f32;/* tile of the single-precision products                  [1]   */
  int32_t cmul;         /* real products per complex double product: 4, or 3 by
                           Gauss's method (3/4 of the matrix-core work; error
                           bounded normwise, not componentwise)  [4]   */
  int32_t dense_coupling; /* 1: multiply the coupling blocks A_{i,i+1} as dense
                           blocks; otherwise products with a coupling operand
                           skip its zero 16 x 16 slabs (zero in both H_{i,i+1} and
                           S_{i,i+1}; exact zeros: the results are the same) [0] */
} negf_options;

/* Operation codes for negf_workspace_bytes. */
enum { NEGF_OP_OBC = 0, NEGF_OP_RETARDED = 1, NEGF_OP_LESSER_GREATER = 2, NEGF_OP_TRANSMISSION = 3 };

/* Bytes of device workspace the call `op` needs for these problems (>= 256-byte
 * aligned pointer expected).  With opt->batch = B the size covers B points in
 * flight and the call loops over the points in chunks of B. */
size_t negf_workspace_bytes(int32_t op, const negf_problem* problems, int32_t n_prob, negf_precision prec,
                            const negf_options* opt);

/* Open-boundary self-energy of one lead (side 0 = left, 1 = right) at every
 * point: the surface Green's function g_s = (d - alpha g_s beta)^{-1} by
 * Sancho-Rubio decimation with z = E + i eta, d = z S0 - H0,
 * alpha = H1 - z S1, beta = H1^H - z S1^H (H1, S1: coupling from the surface
 * cell to the next cell away from the device), and Sigma^R = alpha g_s beta.
 * This is the boundary term of B^R in Eq. (1).
 *  seed     : NULL, or [points][b][b] initial guesses g~ (learned initialiser,
 *             Section IV): the candidate g0 = (d - alpha g~ beta)^{-1} is
 *             accepted when its normalised residual is <= sr_accept; else the
 *             decimation runs, and after every step k the chain is closed
 *             with the seed, X = (eps_k - eps_s,k + d - alpha g~ beta)^{-1},
 *             g^ = (eps_s,k - a_k X c_k)^{-1} (exact for g~ = g_s), which is
 *             accepted at the first k whose residual is <= sr_accept; else the
 *             plain result.  Each closure costs two inversions and five
 *             products per step.
 *  g_surf   : out [points][b][b]; sigma_r: out [points][b][b]
 *  iters    : out int32 [points] decimation steps (0 when the candidate was
 *             accepted, k when the closure after step k was; -k when the
 *             couplings' norms after step k were not finite, which stopped
 *             that point's decimation there)
 *  resid    : out double [points] ||(d - alpha g_s beta) g_s - I||_F /
 *             (||d - alpha g_s beta||_F ||g_s||_F)
 *  info     : out int32 [points]                                              */
negf_status negf_obc_surface(const negf_problem* problems, int32_t n_prob, int32_t side, const negf_options* opt,
                             const void* seed, void* g_surf, void* sigma_r, int32_t* iters, double* resid,
                             int32_t* info, void* workspace, size_t ws_bytes, void* stream);

/* Retarded Green's function, Eq. (1), by RGF: the diagonal blocks
 * GR_diag [points][nb][b][b], the upper blocks G_{i,i+1} GR_upper
 * [points][nb-1][b][b] and (optional, NULL to skip) the lower blocks
 * G_{i+1,i} GR_lower [points][nb-1][b][b].  Both leads are solved inside. */
negf_status negf_rgf_retarded(const negf_problem* problems, int32_t n_prob, negf_precision prec,
                              const negf_options* opt, void* GR_diag, void* GR_upper, void* GR_lower, int32_t* info,
                              void* workspace, size_t ws_bytes, void* stream);

/* Retarded plus lesser (and optionally greater) Green's functions, Eq. (1)
 * and Eq. (2) with B^<> = Sigma^<>_B + Sigma^<>_sc.  GR_* as above (GR_lower
 * may be NULL); GL_diag [points][nb][b][b] and GL_upper [points][nb-1][b][b]
 * (G^<_{i,i+1}; the lower blocks are -(G^<_{i,i+1})^H) are required;
 * GG_diag / GG_upper (greater) may both be NULL to skip G^>. */
negf_status negf_rgf_lesser_greater(const negf_problem* problems, int32_t n_prob, negf_precision prec,
                                    const negf_options* opt, void* GR_diag, void* GR_upper, void* GR_lower,
                                    void* GL_diag, void* GL_upper, void* GG_diag, void* GG_upper, int32_t* info,
                                    void* workspace, size_t ws_bytes, void* stream);

/* ---- allocation-free variant, for callers that cannot allocate device
 * memory or pass a workspace: code under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc. ----
 * negf_rgf_lesser_greater without the workspace arguments: the scratch is a
 * file-scope device array of NEGF_STATIC_SCRATCH_BYTES inside the library, one
 * copy per GPU, reserved when the library's code is first used on that GPU
 * and held until the process ends.  The call allocates nothing (no hipMalloc,
 * no library that allocates).  Points are processed in chunks of opt->batch
 * points, or, when opt->batch is 0, of the largest number whose workspace
 * (negf_workspace_bytes with that batch) fits the scratch.  Returns
 * NEGF_ENOMEM synchronously, enqueueing nothing, when one point (or the
 * requested batch) does not fit: e.g. Nb = 60 blocks of b = 512 need
 * ~368 MiB per point and are rejected; Nb = 60 blocks of b = 128 take 10
 * points per chunk.  Every other argument, output and error as for
 * negf_rgf_lesser_greater.  All calls on one GPU share the one scratch
 * array, which keeps whatever the last call left (nothing of it is read
 * before it is written): calls that may overlap on one GPU (other host
 * threads, other streams) race and must be serialised by the caller. */
#define NEGF_STATIC_SCRATCH_BYTES (256u << 20)
negf_status negf_rgf_lesser_greater_static(const negf_problem* problems, int32_t n_prob, negf_precision prec,
                                           const negf_options* opt, void* GR_diag, void* GR_upper, void* GR_lower,
                                           void* GL_diag, void* GL_upper, void* GG_diag, void* GG_upper,
                                           int32_t* info, void* stream);

/* Transmission T(E) = Tr[Gamma_R G_{N-1,0} Gamma_L G_{N-1,0}^H] per point
 * (double [points]); G_{N-1,0} from the left-connected recursion of the RGF
 * forward sweep.  This is the observable of the paper's Fig. 7. */
negf_status negf_transmission(const negf_problem* problems, int32_t n_prob, const negf_options* opt, double* T,
                              int32_t* info, void* workspace, size_t ws_bytes, void* stream);

/* ---- partitioned selected inversion (Serinv): one device split into
 * partitions that are eliminated in parallel (Fig. 3 and the paragraph after
 * it in Section II) ----
 * The same outputs as negf_rgf_lesser_greater for ONE problem (a device and
 * its energies), computed by splitting the nb blocks into `partitions`
 * partitions of period T = ceil((nb + 1) / partitions): each partition
 * eliminates its interior blocks independently (partitions and energies are
 * one batch axis), the 2 (partitions - 1) boundary blocks form a reduced
 * block-tridiagonal system (retarded and lesser/greater Schur complements)
 * solved sequentially, and each partition then recovers its selected blocks
 * with the boundary self-energies the reduced system gives.  This fills the
 * GPU with `partitions` times more work per launch when few energies are
 * solved at once.  Plain double precision (opt->cmul and tile/panel knobs
 * apply; the decimation as in negf_rgf_lesser_greater).
 * Requirements: partitions >= 2, T >= 3 and nb - (partitions - 1) T >= 1,
 * else NEGF_EINVAL.  GR_lower may be NULL; GG_diag / GG_upper both NULL skip
 * G^>.  Workspace: negf_serinv_workspace_bytes(problem, partitions, greater). */
size_t negf_serinv_workspace_bytes(const negf_problem* problem, int32_t partitions, int32_t greater);
negf_status negf_serinv_lesser_greater(const negf_problem* problem, int32_t partitions, const negf_options* opt,
                                       void* GR_diag, void* GR_upper, void* GR_lower, void* GL_diag, void* GL_upper,
                                       void* GG_diag, void* GG_upper, int32_t* info, void* workspace, size_t ws_bytes,
                                       void* stream);

/* ---- energy convolution of Eq. (3) and the energy/element layout change ----
 * Eq. (3) builds a self-energy from an integral over energy of an element-wise
 * product, B(E) ~ int dE' C1(E - E') (.) C2(E') (M1 = M2 = I, the GW form);
 * the paper evaluates it with FFTs (Section II, after Fig. 3).  On a uniform
 * grid, for every element x of energy-major complex128 arrays
 * G [n_e][n_el], W [n_w][n_el] (W[k] at frequency (k - k0) dE):
 *     B[e][x] = scale * sum_{k=0}^{n_w-1} G[e + k0 - k][x] * W[k][x]
 * with G zero outside [0, n_e); scale (host, 2 doubles) carries dE and the
 * prefactor.  Computed per element by zero-padded FFTs of length
 * L = 2^max(4, ceil(log2(n_e + n_w - 1))), held in registers (LDS carries
 * only the exchanges between radix-8 passes), reading and writing the
 * energy-major layout directly.  Requirements: n_e, n_w >= 1, 0 <= k0 < n_w,
 * n_e + n_w - 1 <= 4096; B must not overlap G or W.  Workspace (twiddles):
 * negf_econv_workspace_bytes(n_e, n_w).  Errors: EINVAL, EHIP. */
size_t negf_econv_workspace_bytes(int32_t n_e, int32_t n_w);
negf_status negf_energy_convolution(int32_t n_e, int64_t n_el, const void* G, int32_t n_w, int32_t k0, const void* W,
                                    const double* scale, void* B, void* workspace, size_t ws_bytes, void* stream);
/* The (E; i,j) <-> (i,j; E) layout change of Fig. 2 on one GPU:
 * dst[c][r] = src[r][c] for a rows x cols complex128 array (dst must not
 * overlap src).  Errors: EINVAL, EHIP. */
negf_status negf_transpose(int64_t rows, int64_t cols, const void* src, void* dst, void* stream);

/* ---- observables of Section III from the outputs of the sweeps ----
 * Per point of the problems (outputs laid out as negf_rgf_lesser_greater
 * writes them):
 *   dos[point][i]     = -Im Tr G^R_ii / pi                      (the block-resolved density of states)
 *   current[point][i] = -2 Re Tr[A_{i,i+1} G^<_{i+1,i}]         (i < nb - 1; e = hbar = 1, one spin)
 * with A_{i,i+1} = E S_{i,i+1} - H_{i,i+1} and G^<_{i+1,i} = -(G^<_{i,i+1})^H,
 * i.e. 2 Re sum_ab A_{i,i+1}[a][b] conj(G^<_{i,i+1}[a][b]).  The spectral
 * current is the same at every interface when the current is conserved (the
 * paper's check of its implementation, Section III).  GR_diag is needed for
 * dos, GL_upper for current; either output may be NULL.  Device doubles,
 * point-major, problems in order.  Errors: EINVAL (a required pointer
 * missing or misaligned, more than 65535 energies in a problem), EHIP. */
negf_status negf_observables(const negf_problem* problems, int32_t n_prob, const void* GR_diag, const void* GL_upper,
                             double* dos, double* current, void* stream);

/* ---- the self-consistent loop of Fig. 1 (Eq. (1)-(3)) with a fixed boson bath ----
 * Alternates the two halves of Fig. 1 for n_prob >= 1 problems, one per
 * transverse momentum k (devices H(k) of one block shape, each with the same
 * n_e >= 1 energies on a uniform grid of spacing dE): every energy is solved from
 * Eq. (1) and (2) with its own block-diagonal scattering self-energies, then
 * the self-energies are rebuilt from the new G^<> by the energy convolution
 * of Eq. (3), restricted to the diagonal blocks:
 *     F^<>_ii(E_e) = scale * sum_k G^<>_ii(E_e - w_k) (.) W^<>[k],  w_k = (k - k0) dE
 * (with several k-points G^<> here is the average over them of each energy:
 * the self-energies are taken independent of k)
 * (M1 = M2 = I; W^<> [n_w][nb][b][b] complex128, a bath held fixed: the
 * polarisation loop of Fig. 1 is not run; scale, host, 2 doubles, e.g.
 * i dE / 2 pi).  The retarded self-energy is (Sigma^> - Sigma^<) / 2 (its
 * principal-value part is not formed).  Iteration n solves with Sigma_n and
 * measures r_n = ||F - Sigma_n||_F / ||F||_F over both kinds, every energy
 * and block (0 when both norms are 0); it stops when r_n <= tol or at
 * n = max_iter - 1, leaving Sigma_n and the Green's functions it produced in
 * the outputs, else, with memory = 0, Sigma_{n+1} = Sigma_n + mixing
 * (F - Sigma_n) (both kinds), and Sigma^R_{n+1} = (Sigma^>_{n+1} -
 * Sigma^<_{n+1}) / 2.  With memory M in 1..4 the update is Anderson's (Pulay's)
 * extrapolation instead: x = (Sigma^<, Sigma^>), f = F - x, dx_j and df_j the
 * differences of the last k = min(n, M) consecutive pairs (x, f), gamma the
 * solution of A gamma = r with A_ij = Re <df_i, df_j> (diagonal raised by
 * 1e-12 trace(A) / k) and r_i = Re <df_i, f_n>, and
 * x_{n+1} = x_n + mixing f_n - sum_j gamma_j (dx_j + mixing df_j); it
 * converges where linear mixing diverges on some devices, at the cost of
 * 2 M + 2 more [n_e][nb][b][b] pairs of workspace (a singular A, df all zero,
 * gives a non-finite Sigma and NEGF_ENONFINITE at the next residual).
 * problem[n_prob]: devices without scattering self-energies and sc_stride 0
 * (the loop supplies both).  sig_r / sig_l / sig_g: device,
 * [n_e][nb][b][b] complex128, in: Sigma_0 (sig_r is overwritten from sig_l
 * and sig_g before the first solve), out: the final Sigma_n.  Outputs as in
 * negf_rgf_lesser_greater for the n_prob problems (point-major, problems in
 * order; GR_lower may be NULL; G^> is required), info [n_prob n_e] per point
 * of the last solve.  n_iter (host): solves performed;
 * history (host, nullable, max_iter doubles): r_0 .. r_{n_iter-1}.
 * negf_scba drives negf_scba_step from the host and synchronises `stream` once
 * per iteration to read the loop state (the stopping decision), so it cannot
 * be captured in a graph; negf_scba_step can.
 * Requirements: 0 <= k0 < n_w, n_e + n_w - 1 <= 4096, 0 < mixing <= 1, 0 <= memory <= 4,
 * tol >= 0, max_iter >= 1.  Returns NEGF_OK when r_n <= tol was reached,
 * NEGF_ENOCONV when max_iter solves ended above tol, NEGF_ENONFINITE when r_n
 * is not finite (the outputs then hold that iteration); argument errors
 * (EINVAL) before any work.  Workspace: negf_scba_workspace_bytes(...). */
size_t negf_scba_workspace_bytes(const negf_problem* problems, int32_t n_prob, negf_precision prec,
                                 const negf_options* opt, int32_t n_w, int32_t memory);
/* One iteration of that loop, enqueued on `stream` with no host
 * synchronisation (capturable in a graph); arguments as for negf_scba plus:
 * it: the iteration index (it = 0 starts a loop: the state is reset and
 * Sigma^R formed from sig_l, sig_g; with memory > 0 the iterations of a loop
 * are it = 0, 1, 2, ... in order, each but the last with update = 1, since
 * the Anderson history kept in the workspace counts on it); update: 0 = never mix (the last
 * iteration of a fixed count, so that the outputs hold Sigma_n and the Green's
 * functions it produced); history: nullable device array, history[it] = r_it;
 * state: device int32[2], [0] = solves performed until r <= tol (or so far),
 * [1] = 0 running, 1 converged, 2 non-finite residual.  Once [1] != 0 the
 * self-energies are no longer changed, so further iterations recompute the
 * same Green's functions (a fixed number of iterations ends where a loop
 * stopped at convergence ends).  With memory = 0 the workspace
 * (negf_scba_workspace_bytes) holds only one iteration's temporaries, so any
 * workspace of that size serves any iteration; with memory > 0 it also holds
 * the Anderson history, which belongs to one loop.  The loop's state and
 * r history live in caller memory.
 * The iterations of a loop go on one stream in order; calls that overlap on
 * one workspace or one state race.  Errors: EINVAL (as negf_scba, it < 0,
 * state NULL or misaligned), EHIP. */
negf_status negf_scba_step(const negf_problem* problem, int32_t n_prob, negf_precision prec, const negf_options* opt,
                           int32_t n_w, int32_t k0, const void* W_lesser, const void* W_greater,
                           const double* scale, double mixing, int32_t memory, double tol, int32_t it,
                           int32_t update, void* sig_r, void* sig_l, void* sig_g, void* GR_diag, void* GR_upper, void* GR_lower, void* GL_diag,
                           void* GL_upper, void* GG_diag, void* GG_upper, int32_t* info, double* history,
                           int32_t* state, void* workspace, size_t ws_bytes, void* stream);
negf_status negf_scba(const negf_problem* problem, int32_t n_prob, negf_precision prec, const negf_options* opt,
                      int32_t n_w, int32_t k0, const void* W_lesser, const void* W_greater, const double* scale,
                      double mixing, int32_t memory, double tol, int32_t max_iter, void* sig_r, void* sig_l,
                      void* sig_g,
                      void* GR_diag, void* GR_upper, void* GR_lower, void* GL_diag, void* GL_upper, void* GG_diag,
                      void* GG_upper, int32_t* info, int32_t* n_iter, double* history, void* workspace,
                      size_t ws_bytes, void* stream);

/* ---- plans: many problems of uneven block shapes in one launch ----
 * A plan groups the points of all problems into chunks of one block shape
 * (at most `batch` points each, per shape from `tunings`), assigns chunks to
 * n_streams worker streams by estimated work (longest first), and runs the
 * lesser/greater computation of negf_rgf_lesser_greater for all of them; each
 * stream runs its chunks shortest first (the same total, earlier completion
 * of the small ones).
 * The decimation runs a fixed number of steps (opt->sr_max_iter, 40 when 0)
 * with converged points masked out, so a plan never synchronises with the
 * host and can be captured: with use_graph = 1 the first execute captures each
 * worker stream's chunks into a hipGraph of its own, and every execute with the
 * same pointers forks from `stream` to the worker streams, launches each graph on
 * its stream and joins back (energies are read from the problems' device arrays
 * at replay time, so they may be updated in place between replays).  A failed
 * capture returns NEGF_EHIP and leaves no graph behind.
 * The plan is a host object; it creates its worker streams (default priority)
 * and events on first execute and allocates no device memory. */
typedef struct negf_plan negf_plan;
typedef struct negf_tuning {
  int32_t b;          /* block size this entry applies to */
  int32_t gemm_tile;  /* as negf_options.gemm_tile (0: default) */
  int32_t gemm_tile_f32;
  int32_t inv_nb;     /* 16 or 32 (0: default) */
  int32_t batch;      /* points per chunk (0: all points of the shape) */
} negf_tuning;
negf_status negf_plan_create(const negf_problem* problems, int32_t n_prob, negf_precision prec,
                             const negf_options* opt, const negf_tuning* tunings, int32_t n_tunings,
                             int32_t n_streams, negf_plan** plan);
size_t negf_plan_workspace_bytes(const negf_plan* plan);
/* Number of chunks; fills (if non-NULL) each chunk's first point index, point
 * count and stream index. */
int32_t negf_plan_chunks(const negf_plan* plan, int32_t* first_point, int32_t* n_points, int32_t* stream_index);
/* Outputs as for negf_rgf_lesser_greater.  stamps (nullable): device uint64
 * [chunks + 1]; stamps[0] = wall clock at the start, stamps[1 + c] = when
 * chunk c finished (ticks of negf_plan_clock_hz()). */
negf_status negf_plan_execute(negf_plan* plan, int32_t use_graph, void* GR_diag, void* GR_upper, void* GR_lower,
                              void* GL_diag, void* GL_upper, void* GG_diag, void* GG_upper, int32_t* info,
                              uint64_t* stamps, void* workspace, size_t ws_bytes, void* stream);
double negf_plan_clock_hz(void);
void negf_plan_destroy(negf_plan* plan);

/* ---- point queue: task lists streamed through a plan (Section II: the
 * energies are independent and are solved in parallel) ----
 * Problem q of the plan provides n_e slots: its energies array, which the queue
 * rewrites (caller-owned device memory).  Its task list task_E[q] (device,
 * n_tasks[q] doubles; task_E and n_tasks are host arrays over the problems) holds
 * the energies to solve.  negf_plan_run_queue forks to the plan's worker streams
 * and runs rounds there: in a round each chunk first takes its slots' next
 * tasks from a device-side round counter (in round r, slot i of problem q takes
 * task r n_e[q] + i; a slot past the end of the list keeps its energy, runs
 * again and reports nothing), then runs as in negf_plan_execute, then writes for
 * every task it solved: task_info, task_dos = -Im sum_k Tr G^R_kk / pi (the
 * oracle's block-resolved density of states, summed) and task_stamps = the wall
 * clock (ticks of negf_plan_clock_hz()) when the chunk finished.  Results are
 * concatenated over the problems in problem order (sum n_tasks entries each).
 * A worker stream runs as many rounds as the problems of its chunks need
 * (the largest ceil(n_tasks[q] / n_e[q])); streams do not wait for each other
 * between rounds.  With use_graph = 1 each worker stream's round is captured once
 * (again when any pointer or task count changes) and replayed.  start_stamp
 * (nullable, device uint64) receives the wall clock before the first round.
 * queue_ws: caller-owned device memory of negf_plan_queue_bytes(plan) bytes
 * (round counters, the slots' current tasks).  The outputs hold the last round's
 * points.  Enqueued only (no host synchronisation); the caller synchronises
 * `stream` before reading results.  Errors: EINVAL (arguments, including tasks
 * for a problem with no slots), EHIP. */
size_t negf_plan_queue_bytes(const negf_plan* plan);
negf_status negf_plan_run_queue(negf_plan* plan, int32_t use_graph, const double* const* task_E,
                                const int32_t* n_tasks, int32_t* task_info, double* task_dos, uint64_t* task_stamps,
                                uint64_t* start_stamp, void* GR_diag, void* GR_upper, void* GR_lower, void* GL_diag,
                                void* GL_upper, void* GG_diag, void* GG_upper, int32_t* info, void* queue_ws,
                                size_t queue_bytes, void* workspace, size_t ws_bytes, void* stream);

/* ---- kernel-level entry points (used by the tests and the tile tuner) ---- */

/* C_p = alpha op(A_p) op(B_p) + beta C_p for p < batch, complex128 M x N
 * outputs, op = 'N' or 'C' (conjugate transpose).  lda/ldb/ldc are row
 * strides, sa/sb/sc batch strides, all in complex elements.  alpha, beta:
 * host arrays of 2 doubles.  prec: 0 double, 1 single products, 2 double
 * with three real products per complex product (Gauss's method); adding 4
 * declares the result anti-Hermitian (M == N): only its upper triangle is
 * computed and the strict lower triangle is set to -conj of the upper one.
 * tile: 0 default, 1 = 64x64, 2 = 128x64, 3 = 128x128, 4 = 64x64 (8 waves),
 * 5 = 128x64 (16 waves), 6 = 32x32 output tiles (taken as given here).
 * Returns NEGF_EINVAL for bad sizes. */
negf_status negf_zgemm_batched(char opa, char opb, int32_t M, int32_t N, int32_t K, const double* alpha,
                               const void* A, int64_t lda, int64_t sa, const void* B, int64_t ldb, int64_t sb,
                               const double* beta, void* C, int64_t ldc, int64_t sc, int32_t batch, int32_t prec,
                               int32_t tile, void* stream);

/* out_p = M_p^{-1} for n x n complex128 blocks (contiguous, batch stride n*n).
 * M is overwritten.  info [batch] receives ESINGULAR / ENONFINITE.
 * workspace: negf_inverse_workspace_bytes(n, batch) bytes.  nb: 16 or 32. */
size_t negf_inverse_workspace_bytes(int32_t n, int32_t batch);
negf_status negf_zinv_batched(int32_t n, int32_t batch, void* M, void* out, int32_t* info, int32_t nb,
                              void* workspace, size_t ws_bytes, void* stream);

/* ---- learned lead initialiser (small MLP, see the seed argument of
 * negf_obc_surface).  Three linear layers X[n][F] -> H -> H -> O with tanh
 * after the first two; weights W1 [F][H], W2 [H][H], W3 [H][O] and biases
 * b1 [H], b2 [H], b3 [O], all float32 row-major device arrays.  Training
 * runs in single precision; inference in bfloat16 (uint16 bit patterns) with
 * single-precision accumulation.  Errors: EINVAL for bad sizes or null
 * pointers, EHIP for launch failures. ---- */

/* Forward pass; keeps the activations A1, A2 [n][H] for the backward pass. */
negf_status negf_mlp_forward(int32_t n, int32_t F, int32_t H, int32_t O, const float* X, const float* W1,
                             const float* b1, const float* W2, const float* b2, const float* W3, const float* b3,
                             float* A1, float* A2, float* Y, void* stream);
/* Gradients of L = mean over n*O entries of (Y - T)^2 with respect to every
 * parameter.  dY [n][O], dZ2 [n][H], dZ1 [n][H] are caller scratch. */
negf_status negf_mlp_backward(int32_t n, int32_t F, int32_t H, int32_t O, const float* X, const float* W2,
                              const float* W3, const float* A1, const float* A2, const float* Y, const float* T,
                              float* dW1, float* db1, float* dW2, float* db2, float* dW3, float* db3, float* dY,
                              float* dZ2, float* dZ1, void* stream);
/* One Adam step (bias-corrected, step t >= 1) on a flat parameter array. */
negf_status negf_mlp_adam_step(int32_t count, float* param, const float* grad, float* m, float* v, int32_t t,
                               float lr, float beta1, float beta2, float eps, void* stream);
/* Round float32 to bfloat16 (nearest even). */
negf_status negf_mlp_to_bf16(const float* src, uint16_t* dst, int64_t count, void* stream);
/* bfloat16 inference: Xb [n][F], W*b bf16 weights, float biases, Y [n][O]
 * float32; scratch holds 2*n*H bf16 activations. */
negf_status negf_mlp_infer_bf16(int32_t n, int32_t F, int32_t H, int32_t O, const uint16_t* Xb, const uint16_t* W1b,
                                const float* b1, const uint16_t* W2b, const float* b2, const uint16_t* W3b,
                                const float* b3, uint16_t* scratch, float* Y, void* stream);

/* Data transforms of the learned pipeline (the network's input features are
 * standardised, its targets compressed; Section IV's learned shortcut, built
 * here as the seed of the lead decimation).  float32 row-major arrays.
 *  negf_mlp_moments : mu[c] = mean over the n rows of X[r][c], sd[c] = the
 *                     sample standard deviation (n - 1), at least 1e-6;
 *                     accumulated in double; scratch: 65 * F doubles.
 *  negf_mlp_normalize: Xn[r][c] = (X[r][c] - mu[c]) / sd[c] (Xn may be X).
 *  negf_mlp_signed_log: y = sign(x) log(1 + |x|), or with inverse = 1 its
 *                     inverse sign(x) (exp(|x|) - 1) (y may be x).
 *  negf_mlp_mse     : *out = mean over count entries of (Y - T)^2 (double);
 *                     scratch: 64 doubles.
 * Mode transforms of the per-mode seed (complex128 [n][b][b] blocks):
 *  negf_mode_diag   : out[p * b + j] = (Re, Im) of T_p[j][j] as float pairs.
 *  negf_mode_scale_columns: out_p = U diag(x_p), x_p[j] = y[p * b + j][0] +
 *                     i y[p * b + j][1] (U [b][b], y float pairs), i.e. the
 *                     left factor of the seed U diag(x) U^H.
 * Errors: EINVAL for bad sizes or null pointers, EHIP for launch failures. */
negf_status negf_mlp_moments(int64_t n, int32_t F, const float* X, float* mu, float* sd, double* scratch,
                             void* stream);
negf_status negf_mlp_normalize(int64_t n, int32_t F, const float* X, const float* mu, const float* sd, float* Xn,
                               void* stream);
negf_status negf_mlp_signed_log(int64_t count, const float* x, float* y, int32_t inverse, void* stream);
negf_status negf_mlp_mse(int64_t count, const float* Y, const float* T, double* out, double* scratch, void* stream);
negf_status negf_mode_diag(int32_t n, int32_t b, const void* T, float* out, void* stream);
negf_status negf_mode_scale_columns(int32_t n, int32_t b, const void* U, const float* y, void* out, void* stream);

/* ---- profiling: per kernel class launch counts, executed flops and
 * event-timed durations, recorded on the launching stream.  Flops are those
 * the kernels execute: 6 M N K per complex product in Gauss's three-product
 * form, 8 M N K with four real products, 8 n w^2 per inversion panel of width
 * w.  What a launch executes depends on device data (the decimation masks
 * converged pairs out of later steps; NEGF_KC_GEMM_CPL, the products with a
 * coupling-block operand, skip its zero slabs), so the kernels count their
 * own flops into device counters while profiling is on (one set per process,
 * on the device current when profiling was enabled). ---- */
enum { NEGF_KC_GEMM64 = 0, NEGF_KC_GEMM32 = 1, NEGF_KC_INV_PANEL = 2, NEGF_KC_INV_SWAP = 3, NEGF_KC_INV_PERM = 4,
       NEGF_KC_ELEM = 5, NEGF_KC_INV_GEMM = 6, NEGF_KC_GEMM_CPL = 7, NEGF_KC_COUNT = 8 };
typedef struct negf_kernel_stats {
  int64_t launches;
  double total_ms;   /* sum of per-launch event durations */
  double flops;      /* real flops the matrix cores executed in those launches */
  double bytes;      /* algorithmic HBM bytes of those launches */
} negf_kernel_stats;
/* Enable (1) / disable (0) timing; enabling resets the counters (and
 * synchronises with the device to clear the instruction counter).  Timing
 * pairs events around each launch; counters are read after the caller has
 * synchronised every stream it used. */
void negf_profile_enable(int32_t on);
/* Which kernel classes get timing events while profiling is on: bit k set
 * times class k (default: all).  Every event pair costs host time per launch,
 * so a run that times one class (the products, ~4 % of the launches of an RGF
 * call) keeps close to the unprofiled speed; the flop counters cover every
 * class regardless (launches and total_ms stay 0 for untimed classes). */
void negf_profile_time_classes(uint32_t mask);
/* Fill stats[NEGF_KC_COUNT]; returns NEGF_EHIP if an event query failed. */
negf_status negf_profile_read(negf_kernel_stats* stats);

const char* negf_status_string(negf_status s);
/* 101: negf_problem carries sc_stride (energy-dependent scattering
 * self-energies); callers built against 100 pass a shorter struct.
 * 102: the loop's entry points take the Anderson memory. */
int32_t negf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NEGF_H */
