/*
 * rgf.h — C ABI of the MI355X (gfx950) recursive Green's function library.
 *
 * The library computes the selected inverse bndiag(M^{-1}) of the block n-diagonal
 * matrix M(E) = (E + i*eta_d) I - H - Sigma_L(E) (+) Sigma_R(E) for many energies E
 * (paper "Revisiting recursive methods for Dyson and Keldysh in NEGF: Part I",
 * Sec. 2 introduction: the Dyson problem is to extract the block n-diagonal part
 * of the inverse of the block n-diagonal matrix M), and the transmission
 *     T(E) = Re Tr[Gamma_L G_{0,l-1} Gamma_R G_{0,l-1}^H],  Gamma = i (Sigma - Sigma^H).
 * Two methods: the sequential Schur-complement sweep (Sec. 2.2 Algorithm 1 for
 * w = 1, Sec. 2.3 for w > 1) and domain-decomposition RGF (Sec. 3, Algorithm 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Complex numbers are interleaved pairs of double (the torch.complex128 layout).
 *    Every b x b block is row-major and contiguous.
 *  - Layers are numbered 0..l-1.  A block band of half-bandwidth w is stored as
 *    X[2w+1][l][b][b] where X[w+k][i] is the block (i, i+k), k in [-w, w]; blocks
 *    with i+k outside [0, l) are never read and never written.
 *  - H: the band of the device Hamiltonian, shared by all energies (device memory).
 *    H is not assumed Hermitian.  sigma_L / sigma_R: [nE][b][b] retarded lead
 *    self-energies (device memory), attached to layer 0 and layer l-1; they
 *    already include the lead's own broadening.  energies: [nE] doubles (device).
 *  - G: output band [nE][2w+1][l][b][b] (device).  T: [nE] doubles (device),
 *    may be NULL.  info: [nE] int32 (device): 0 = ok; j+1 = layer j held the first
 *    Schur pivot (in elimination order) that was exactly singular or non-finite;
 *    every output of that energy is then set to NaN.
 *  - Ownership: the caller allocates and owns every input, output and workspace;
 *    a plan owns only host metadata.  Solve calls allocate nothing, never
 *    synchronise the stream and return as soon as the work is queued.
 *  - stream is a hipStream_t (NULL = the default stream).
 *  - Errors: argument and plan errors are returned synchronously; numerical
 *    failures are reported per energy through info[] (read after a stream sync).
 *    No entry point aborts or throws.
 *  - A plan is immutable after creation and may be used concurrently on different
 *    streams with distinct workspaces.
 */
#ifndef RGF_MI355X_H
#define RGF_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rgf_plan_s* rgf_plan_t;

typedef enum {
  RGF_OK = 0,
  RGF_ERR_INVALID_ARG = 1,
  RGF_ERR_UNSUPPORTED = 2,
  RGF_ERR_OUT_OF_MEMORY = 3,
  RGF_ERR_WORKSPACE_TOO_SMALL = 4,
  RGF_ERR_HIP = 5,
  RGF_ERR_PLAN_MISMATCH = 6
} rgf_status_t;

typedef enum {
  RGF_FP64 = 0,          /* every product and pivot in FP64 */
  RGF_MIXED_FP32 = 1,    /* every block product on FP32 MFMA (operands rounded to FP32,
                            FP32 accumulation, widened to FP64), Schur pivots inverted in
                            FP64 and refined once in FP64: g <- g + g (I - S g).
                            The FP32 rounding (2^-24) is amplified by the pivots'
                            conditioning, so each energy runs with FP32 products only while
                            every Schur pivot S_i satisfies kappa_1(S_i) * 2^-24 <=
                            mixed_tolerance (desc field; 1e-5 when 0); at the first pivot
                            that does not, the energy is recomputed with FP64 products and
                            RGF_INFO_FP64_PRODUCTS is set in its info entry.
                            Sequential method with w = 1 only (else RGF_ERR_UNSUPPORTED):
                            DDRGF's closed interiors are ill-conditioned at most energies. */
  RGF_MIXED_BF16X3 = 2   /* not built (always RGF_ERR_UNSUPPORTED): split-BF16 products.
                            They would carry the same FP32 accumulation as RGF_MIXED_FP32,
                            whose accuracy is already limited by pivot conditioning. */
} rgf_precision_t;

/* Flag in info[e] after a RGF_MIXED_FP32 solve: energy e was recomputed with FP64
 * products (a Schur pivot was too ill-conditioned for FP32 products).  The low 30
 * bits keep the status described above (0 = ok). */
#define RGF_INFO_FP64_PRODUCTS 0x40000000
#define RGF_INFO_STATUS_MASK 0x3fffffff

/* Status bit in info[e] of a sequential solve run with several workgroups per
 * energy (rgf_plan_set_split): a workgroup of that energy gave up waiting for the
 * others at a group barrier.  That energy's outputs are undefined (T is NaN).  Not
 * expected in practice (the launch is cooperative, so every workgroup is resident);
 * it bounds the wait if one is ever missing. */
#define RGF_INFO_SYNC_TIMEOUT 0x20000000

/* want_backward flags */
#define RGF_BACKWARD_ONSITE 1   /* on-site energy gradient */
#define RGF_BACKWARD_BAND 2     /* gradient with respect to the whole band of H (sizes the workspace) */

typedef enum {
  RGF_METHOD_SEQUENTIAL = 0,  /* Schur-complement sweep, Algorithm 1 / Sec. 2.3 */
  RGF_METHOD_DDRGF = 1        /* domain decomposition, Algorithm 2 */
} rgf_method_t;

/* Problem description (host memory). */
typedef struct {
  int64_t num_layers;        /* l >= 1 */
  int64_t block_size;        /* b, 1 <= b <= 128 */
  int64_t half_bandwidth;    /* w >= 1 (1 = block tridiagonal); w < l */
  int64_t num_energies;      /* nE >= 1 */
  int32_t precision;         /* rgf_precision_t */
  int32_t method;            /* rgf_method_t */
  int64_t num_domains;       /* DDRGF: number of (interior, separator) pairs m >= 1 */
  int64_t separator_layers;  /* DDRGF: layers per separator; 0 means w (the only value supported) */
  int32_t want_transmission; /* nonzero: T is computed when the T pointer is not NULL */
  int32_t want_backward;     /* 0, or RGF_BACKWARD_ONSITE and/or RGF_BACKWARD_BAND: rgf_solve keeps
                                the checkpoints rgf_backward needs (sequential, w = 1, FP64) */
  int64_t checkpoint_domains;/* rgf_backward: layers are cut into this many domains (0 = 8) */
  double mixed_tolerance;    /* RGF_MIXED_FP32: largest kappa_1(S_i) * 2^-24 run with FP32
                                products (0 = 1e-5, the mixed-precision error target) */
  int64_t inner_domains;     /* DDRGF, FP64: 0 = the reduced separator system is solved by the
                                sequential sweep; m2 >= 1 = by DDRGF with m2 pairs (two-level
                                recursion of Algorithm 2's step 3); needs num_domains >= 2 m2;
                                w = 1, or w > 1 in the super-block form */
  int64_t ddrgf_form;        /* DDRGF with w > 1: 0 = native n-diagonal interiors (Sec. 2.3 RGF
                                inside each interior, w first and last block rows and columns as
                                halos, reduced system on the m w separator layers as a band of
                                half bandwidth 2w - 1); 1 = w-layer super-block form (w layers
                                become one layer of w b orbitals, then the tridiagonal kernels;
                                needs l % w == 0 and w b <= 128).  Must be 0 otherwise. */
} rgf_desc_t;

/* Validate a description and build a plan.  *workspace_bytes receives the size of
 * the device workspace that rgf_solve / ddrgf_solve need.  Validation: l >= 1,
 * 1 <= b <= 128, 1 <= w, w < l unless l == 1, nE >= 1; DDRGF additionally needs
 * m >= 1 and every interior at least w layers long with separators of w layers
 * (l - m*w >= m*w).  Returns synchronously. */
rgf_status_t rgf_plan_create(const rgf_desc_t* desc, rgf_plan_t* plan, size_t* workspace_bytes);
rgf_status_t rgf_plan_destroy(rgf_plan_t plan);

/* Sequential RGF (Algorithm 1 for w = 1; the n-diagonal sweep of Sec. 2.3 for
 * w > 1) over all energies of the plan.  G, T, info as described above. */
rgf_status_t rgf_solve(rgf_plan_t plan, const void* H, const void* sigma_L, const void* sigma_R,
                       const double* energies, double eta_d, void* G, double* T, int32_t* info,
                       void* workspace, size_t workspace_bytes, void* stream);

/* Lesser Green's function on the band (the Keldysh equation G^< = G^R Sigma^< G^A,
 * the stage after the Dyson equation named in the paper's introduction and
 * outlook).  The lesser self-energies are the leads': Sigma^<_X = i f_X Gamma_X on
 * the layer lead X attaches to, Gamma_X = i (Sigma_X - Sigma_X^H), f_X =
 * occupation_X[e] (DEVICE arrays [nE], e.g. Fermi functions of the leads at each
 * energy); a device broadening eta_d enters G^R only.  Then
 *   G^<_ij = G_{i,0} Sigma^<_L G_{j,0}^H + G_{i,l-1} Sigma^<_R G_{j,l-1}^H,
 * with the first and last block columns of G^R from the multipliers of Algorithm
 * 1's sweep (for w > 1: the first column by the sweep's downward recursion, the last
 * through transfer products of its multipliers, Sec. 2.3).  Runs rgf_solve (same
 * arguments, results and workspace) and then writes G_lesser [nE][2w+1][l][b][b] in
 * the layout of G (blocks outside the matrix are not written; energies whose info is
 * nonzero get NaN).  Sequential FP64 plans without want_backward (else
 * RGF_ERR_UNSUPPORTED). */
rgf_status_t rgf_solve_lesser(rgf_plan_t plan, const void* H, const void* sigma_L, const void* sigma_R,
                              const double* energies, double eta_d, const double* occupation_L,
                              const double* occupation_R, void* G, void* G_lesser, double* T, int32_t* info,
                              void* workspace, size_t workspace_bytes, void* stream);

/* Retarded self-energies of a semi-infinite periodic lead at every energy (the
 * Sigma^r that the selected inversion takes as given input).  The lead repeats
 * principal layers with on-layer block H00 and coupling H01 to the next layer away
 * from the device; its surface Green's function g_s = (z - H00 - H01 g_s H01^H)^{-1},
 * z = E + i eta, is computed by the decimation of Lopez Sancho, Lopez Sancho and
 * Rubio (J. Phys. F 15, 851 (1985)), each step halving the remaining chain, until
 * max|alpha_ij| + max|beta_ij| < tolerance (the couplings of the decimated chain),
 * and sigma[e] = Hc g_s Hc^H with Hc the coupling from the device layer to the lead's
 * surface layer.  H00, H01, Hc: DEVICE [b][b]; energies: DEVICE [nE]; sigma: DEVICE
 * out [nE][b][b] (the layout of sigma_L / sigma_R of rgf_solve); steps: DEVICE out
 * [nE]: the number of decimation steps taken, -1 when max_steps steps did not
 * converge, -2 when a pivot z - eps was singular or non-finite (sigma NaN in both
 * cases).  workspace: rgf_lead_workspace_bytes(b, nE) bytes.  Errors: 1 <= b <= 128,
 * nE >= 1, tolerance > 0, max_steps >= 1, eta >= 0 and non-NULL pointers, else
 * RGF_ERR_INVALID_ARG (b > 128: RGF_ERR_UNSUPPORTED); a smaller workspace gives
 * RGF_ERR_WORKSPACE_TOO_SMALL.  Accuracy: where E + i eta is within ~eta of an
 * eigenvalue of H00 the first steps invert a nearly singular z - eps and the
 * decimation cancels terms of size 1/eta (FP64 loses ~1e-5 at eta = 1e-6). */
rgf_status_t rgf_lead_workspace_bytes(int64_t block_size, int64_t num_energies, size_t* workspace_bytes);
rgf_status_t rgf_lead_self_energy(int64_t block_size, int64_t num_energies, const void* H00, const void* H01,
                                  const void* Hc, const double* energies, double eta, double tolerance,
                                  int32_t max_steps, void* sigma, int32_t* steps, void* workspace,
                                  size_t workspace_bytes, void* stream);

/* Observables read off a solved band (the densities the Dyson and Keldysh stages
 * give, Sec. 1 and the outlook): both read only the diagonal blocks of a band in
 * the layout of G, [nE][2w+1][l][b][b] (DEVICE), and are asynchronous on stream.
 *   rgf_dos:     dos[e][i b + s] = -(1/pi) Im G^R_{ii,ss}(E_e), the orbital-resolved
 *                density of states (DEVICE out [nE][l b]);
 *   rgf_density: density[i b + s] = sum_e weights[e] (1/2pi) Im G^<_{ii,ss}(E_e), the
 *                orbital-resolved electron density by the caller's quadrature weights
 *                (DEVICE [nE], e.g. the energy spacing); energies are summed in order,
 *                so the result is deterministic (DEVICE out [l b]).
 * Errors: l, b, w, nE >= 1 and non-NULL pointers, else RGF_ERR_INVALID_ARG.  NaN
 * entries of an energy whose info is nonzero propagate. */
rgf_status_t rgf_dos(const void* G, int64_t num_layers, int64_t block_size, int64_t half_bandwidth,
                     int64_t num_energies, double* dos, void* stream);
rgf_status_t rgf_density(const void* G_lesser, int64_t num_layers, int64_t block_size, int64_t half_bandwidth,
                         int64_t num_energies, const double* weights, double* density, void* stream);
/* Spectral particle current through every bond (w = 1; hbar = 1, spin not counted):
 * current[e][i] = (1/pi) Re Tr[H_{i,i+1} G^<_{i+1,i}(E_e)], the rate at which charge of
 * layer i flows to layer i+1 per unit energy (from rho = <c^dag c> = -i int dE/2pi G^<).
 * In steady state without device broadening it is the same for every bond and equals
 * T(E) (f_L - f_R) / 2pi.  H: DEVICE band [3][l][b][b] (as for rgf_solve);
 * G_lesser: DEVICE [nE][3][l][b][b] (rgf_solve_lesser); current: DEVICE out
 * [nE][l-1].  Errors: l >= 2, b, nE >= 1 and non-NULL pointers, else
 * RGF_ERR_INVALID_ARG. */
rgf_status_t rgf_bond_current(const void* H, const void* G_lesser, int64_t num_layers, int64_t block_size,
                              int64_t num_energies, double* current, void* stream);

/* Several workgroups per energy for rgf_solve.  With fewer energies than compute
 * units, the sequential sweep (Algorithm 1 for w = 1, the n-diagonal sweep of Sec.
 * 2.3 for w > 1; FP64, plans without want_backward, padded block size 64 or 128)
 * can give each energy K = 2 or 4
 * workgroups: each computes a row slab of every block product, the first also
 * inverts the Schur pivots, and they meet at bounded group barriers (cooperative
 * launch, so all are resident).  Results are bitwise those of one workgroup per
 * energy.  workgroups_per_energy: 0 = the largest K in {4, 2} whose grid fits the
 * device's co-resident capacity (1 when none does), 1 = never split, 2 or 4 = that K
 * when it fits (else 1).  spin_limit: polls of a group barrier before a workgroup
 * gives up (RGF_INFO_SYNC_TIMEOUT); 0 = the default (2^22).  The choice is made at
 * the next solve, on its device; streams under capture always use one workgroup
 * per energy.  Returns RGF_ERR_INVALID_ARG for other values. */
rgf_status_t rgf_plan_set_split(rgf_plan_t plan, int32_t workgroups_per_energy, int64_t spin_limit);

/* Workgroups per energy used by the plan's last rgf_solve (1 before any). */
rgf_status_t rgf_plan_split_workgroups(rgf_plan_t plan, int32_t* workgroups_per_energy);

/* DDRGF (Algorithm 2, one level): interiors of every energy are eliminated
 * independently, separators are stitched through the reduced block-tridiagonal
 * Schur complement (Proposition 4), solved by Algorithm 1, and the band of G is
 * recovered (Algorithm 2, steps 4-5).  For w > 1 (separators of w layers) the
 * interiors run the n-diagonal RGF of Sec. 2.3 and the reduced system is solved
 * by it too (desc ddrgf_form = 0), or everything runs on w-layer super-blocks
 * (ddrgf_form = 1).  Same arguments as rgf_solve; the plan must
 * have been created with method = RGF_METHOD_DDRGF (else RGF_ERR_PLAN_MISMATCH). */
rgf_status_t ddrgf_solve(rgf_plan_t plan, const void* H, const void* sigma_L, const void* sigma_R,
                         const double* energies, double eta_d, void* G, double* T, int32_t* info,
                         void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Batched launch over systems ("devices") of uneven size
 * ---------------------------------------------------------------------------
 * Each device d has its own block-tridiagonal band H_d (l_d layers of b_d orbitals,
 * 1 <= b_d <= 128) and its own energies; one instance = one (device,
 * energy) pair.  All instances run in ONE persistent kernel: workgroups pull
 * instances from a work queue ordered by the plan's schedule and run the whole
 * sweep of each (Algorithm 1); the outputs are T(E) and the diagonal blocks G_ii
 * (the band's off-diagonal blocks are not written).  The first solve on a
 * non-default stream captures the launch into a hipGraph that later solves with the
 * same device table, workspace and stream replay. */

/* Host-side shape of one device. */
typedef struct {
  int64_t num_layers;     /* l_d >= 1 */
  int64_t block_size;     /* b_d in [1, 128] (padded to a multiple of 16 inside) */
  int64_t num_energies;   /* nE_d >= 1 */
} rgf_batch_shape_t;

/* Device-side table entry of one device (the caller fills an array of these in
 * device memory; all pointers are device pointers). */
typedef struct {
  const void* H;            /* band [3][l][b][b] */
  const void* sigma_L;      /* [nE][b][b] */
  const void* sigma_R;      /* [nE][b][b] */
  const double* energies;   /* [nE] */
  void* G_diag;             /* out [nE][l][b][b]: diagonal blocks of G */
  double* T;                /* out [nE], may be NULL */
  int32_t* info;            /* out [nE], as for rgf_solve */
  int32_t num_layers;       /* informational: the kernel takes each device's shape from the plan */
  int32_t block_size;
} rgf_batch_device_t;

typedef enum {
  RGF_SCHEDULE_LONGEST_FIRST = 0,  /* instances by decreasing l*b^3 */
  RGF_SCHEDULE_INPUT_ORDER = 1,    /* device by device, energy by energy */
  RGF_SCHEDULE_INTERLEAVED = 2     /* longest first within each block size, sizes interleaved */
} rgf_schedule_t;

/* Build a batched plan.  shapes: host array [num_devices].  precision: RGF_FP64 or
 * RGF_MIXED_FP32 (with the conditioning switch of RGF_MIXED_FP32 at tolerance 1e-5,
 * reported per instance through RGF_INFO_FP64_PRODUCTS in the device's info[]).
 * schedule: order of the work queue (rgf_schedule_t).  The tile: waves = wave64s
 * per persistent workgroup, 8 (one workgroup per compute unit; 0 means 8) or 4 (two
 * per compute unit, for batches of small blocks); grid = persistent workgroups (0 =
 * one per compute unit of the current device for 8 waves, two for 4).  The
 * schedule, grid and waves of a workload are what the autotuner chooses (the
 * Python binding reads its table).  Unlike the other plans this one owns a small
 * device array (the work queue, 3 ints per instance, and the shapes), allocated
 * here and freed by rgf_plan_destroy; creating it needs a visible GPU.
 * *workspace_bytes: one workspace slot per persistent workgroup, sized for the
 * largest device, plus the queue counter. */
rgf_status_t rgf_batched_plan_create(int64_t num_devices, const rgf_batch_shape_t* shapes,
                                     int32_t precision, int32_t schedule, int32_t grid, int32_t waves,
                                     rgf_plan_t* plan, size_t* workspace_bytes);

/* Run every instance of the plan.  devices: DEVICE array [num_devices] of table
 * entries.  Numerical failures are reported per instance through each device's
 * info[].  Calls on one plan from several host threads are serialised. */
rgf_status_t rgf_batched_solve(rgf_plan_t plan, const rgf_batch_device_t* devices, double eta_d,
                               void* workspace, size_t workspace_bytes, void* stream);

/* Adjoint of the transmission: gradients of L = sum_E dL_dT[E] T(E) with respect to
 * the band of H and to on-site energies (the paper has no gradient; this follows
 * from dG = G dH G, M = (E + i eta_d) I - H - Sigma).
 *
 * With X = Gamma_R G_{0,l-1}^H Gamma_L and Y_ij = G_{j,l-1} X G_{0,i}:
 *   dH[1+k][i] (block (i, j = i+k), k in {-1, 0, 1}) = sum_E dL_dT[E] * 2 Y_ij^H,
 *     the gradient with respect to each entry of H taken as an independent complex
 *     parameter, in PyTorch's convention dL/dRe + i dL/dIm (H is not assumed
 *     Hermitian; blocks outside the matrix are not written);
 *   d_onsite[i][s] = sum_E dL_dT[E] * 2 Re (Y_ii)_ss, the gradient with respect to a
 *     real shift H_ii,ss += eps_{i,s} (the real part of dH's diagonal).
 * The plan must have been created with want_backward (sequential method, w = 1,
 * FP64; RGF_BACKWARD_BAND is needed for dH) and rgf_solve must have run with it on
 * the same H, sigma, energies and eta_d.  Checkpointing: rgf_solve leaves in the
 * first rgf_plan_checkpoint_bytes() bytes of its workspace, per energy and per
 * checkpoint domain, the Schur pivot and the last-column propagator at the domain's
 * last layer and the propagator and first block row at its first layer; only this
 * prefix must be preserved until rgf_backward (the rest of the workspace is scratch
 * for both calls and may be another buffer of the plan's size whose prefix holds a
 * copy).  rgf_backward re-runs each domain's upward sweep from its checkpointed
 * pivot (bitwise the forward's multipliers), one workgroup per (domain, chunk of
 * energies), and sums in a fixed order (deterministic, independent of the domain
 * count).
 * G_diag: diagonal blocks of the forward's G (device), energy e at G_diag + e *
 * g_diag_stride complex elements (0 = l*b*b, i.e. a compact [nE][l][b][b] array; pass
 * G + l*b*b with stride 3*l*b*b to read them from the output band).  dL_dT: [nE]
 * device doubles.  dH: band [3][l][b][b] (device, may be NULL); d_onsite: [l][b]
 * device doubles (may be NULL); not both NULL. */
rgf_status_t rgf_backward(rgf_plan_t plan, const void* H, const void* sigma_L, const void* sigma_R,
                          const double* energies, double eta_d, const void* G_diag, int64_t g_diag_stride,
                          const double* dL_dT, void* dH, double* d_onsite, void* workspace,
                          size_t workspace_bytes, void* stream);

/* Bytes at the start of the workspace that rgf_backward reads from the forward
 * (0 for plans without want_backward). */
rgf_status_t rgf_plan_checkpoint_bytes(rgf_plan_t plan, size_t* checkpoint_bytes);

/* Workspace size of a plan (the value rgf_plan_create returned). */
rgf_status_t rgf_plan_workspace_bytes(rgf_plan_t plan, size_t* workspace_bytes);

/* rgf_solve without a workspace argument, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that forbid
 * allocation).  The workspace is a static device array of the library, 64 MiB
 * (67108864 bytes) per device, held until the process ends; this call allocates
 * nothing.  Plans whose workspace exceeds it are refused
 * with RGF_ERR_WORKSPACE_TOO_SMALL, plans made with want_backward with
 * RGF_ERR_UNSUPPORTED.  All calls on one device share the array: calls that
 * overlap on a device (concurrent streams or host threads) race and must be
 * serialised by the caller.  Other arguments and results as rgf_solve. */
rgf_status_t rgf_solve_noalloc(rgf_plan_t plan, const void* H, const void* sigma_L, const void* sigma_R,
                               const double* energies, double eta_d, void* G, double* T, int32_t* info,
                               void* stream);

/* ---------------------------------------------------------------------------
 * Per-kernel timing (measurement aid; not part of the method).
 *
 * rgf_plan_set_timing(plan, 1, max_marks) creates a pool of max_marks HIP events
 * owned by the plan (host-side creation; call it outside graph capture).  While
 * timing is enabled, rgf_solve, ddrgf_solve and rgf_backward record one event on
 * their stream before their first kernel and one after every kernel they launch,
 * so a kernel's duration is the time between the event before it and the event
 * after it on that stream.  Events beyond the pool are not recorded (the next
 * query reports how many were dropped).  Batched solves are not timed.
 * rgf_plan_set_timing(plan, 0, 0) destroys the pool.  Returns RGF_ERR_INVALID_ARG
 * for a NULL plan or max_marks < 2 when enabling, RGF_ERR_HIP if event creation
 * fails.
 *
 * rgf_plan_kernel_times waits for the last recorded event (the host blocks), sums
 * the durations per kernel name over every solve since the previous query, writes
 * up to max_entries entries in order of first appearance, sets *n_entries to the
 * number of distinct kernels (which may exceed max_entries) and *dropped (may be
 * NULL) to the number of marks lost to a full pool, and empties the pool.
 * Returns RGF_ERR_INVALID_ARG when timing is not enabled or out / n_entries is
 * NULL, RGF_ERR_HIP if an event query fails.  Must not run concurrently with a
 * solve on the same plan.
 * ------------------------------------------------------------------------- */
typedef struct {
  char name[48];       /* kernel name, NUL-terminated */
  double total_ms;     /* summed duration of its launches */
  int64_t launches;    /* number of launches timed */
} rgf_kernel_time_t;

rgf_status_t rgf_plan_set_timing(rgf_plan_t plan, int32_t enable, int32_t max_marks);
rgf_status_t rgf_plan_kernel_times(rgf_plan_t plan, rgf_kernel_time_t* out, int32_t max_entries,
                                   int32_t* n_entries, int32_t* dropped);

/* Static text of a status code. */
const char* rgf_status_string(rgf_status_t status);

/* Library version as 10000*major + 100*minor + patch. */
int rgf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RGF_MI355X_H */
