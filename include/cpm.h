/*
 * cpm.h -- C-ABI of libcpm, the GPU constant-potential electrostatics path.
 *
 * Method: Tee & Searles, "Fully Periodic, Computationally Efficient Constant
 * Potential Molecular Dynamics Simulations of Ionic Liquid Supercapacitors"
 * (arXiv 2201.12963).  Electrode atoms carry Gaussian charges (Eq. 2); the
 * Coulomb energy is the quadratic form U = U_elyt - q.b + 1/2 q.A q (Eq. 3);
 * the electroneutral constant-potential charges are q* = S v with the
 * projected inverse S = O A^-1 (Eq. 8-9) or O1 O A^-1 for the doubled cell
 * (Eq. 14-15), and v = b + dV c with c = d (doubled cell) or d - z/Lz
 * (finite field, Eq. 11 with the lower electrode taken one period up).
 *
 * Units: nm, e, V, eV.  Coulomb constant k_e = 1.43996454784 eV nm / e^2.
 *
 * Conventions for every call:
 *  - Arrays are structure-of-arrays, float64, contiguous.  "device" pointers
 *    are HIP device memory owned by the caller (for instance data_ptr() of a
 *    contiguous torch tensor); "host" pointers are ordinary host memory.
 *  - All work is enqueued asynchronously on the stream given to cpm_create
 *    (or cpm_set_stream).  Nothing blocks unless stated.
 *  - No exception crosses the ABI.  Every int-returning call returns CPM_OK
 *    or a negative status; cpm_last_error() then holds a message.
 *  - A context is not thread-safe.  Calls on one context are ordered by its
 *    stream; two contexts may run concurrently.
 *  - Site positions may lie anywhere: every kernel wraps them into the cell.
 *    Non-finite positions are reported by cpm_sync_status().
 */
#ifndef CPM_H
#define CPM_H

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
enum {
  CPM_OK = 0,
  CPM_EINVAL = -1,     /* bad descriptor or argument */
  CPM_ESTATE = -2,     /* call out of order (e.g. solve before build) */
  CPM_ENOTSPD = -3,    /* elastance matrix not positive definite */
  CPM_EDEVICE = -4,    /* HIP runtime error */
  CPM_ENOMEM = -5,     /* device allocation failed / batch too large */
  CPM_ENONFINITE = -6  /* non-finite input or result */
};

/* geometry (Sec. II.B of the paper).  CPM_SLAB is the mixed-periodicity
 * setting the paper compares against (Fig. 2b): box[2] is the lengthened
 * z period, the electrodes and electrolyte occupy at most half of it with the
 * empty space across z = 0, and the charged-sheet (dipole) correction
 * k_e 2 pi / V M_z^2, M_z = sum q z over all charges, enters A (k_e 4 pi/V
 * z z^T), b (-k_e 4 pi/V z sum_j Q_j Z_j), the electrolyte energy and the
 * site forces (-k_e 4 pi/V Q_j M_z along z); the electrode potentials are
 * psibar e + dV d with one neutrality constraint. */
enum { CPM_FINITE_FIELD = 0, CPM_DOUBLED_CELL = 1, CPM_SLAB = 2 };
/* reciprocal-space method for the electrolyte sums */
enum { CPM_KSPACE_EWALD = 0, CPM_KSPACE_PPPM = 1 };
/* arithmetic of the per-step path: FP64 throughout, or FP32 mesh / FFT /
 * real space with FP32 accumulation (the elastance build, the inversion,
 * the neutrality re-projection and the energy sums stay FP64) */
enum { CPM_FP64 = 0, CPM_MIXED = 1 };

typedef struct cpm_ctx cpm_ctx;

typedef struct {
  double box[3];        /* Lx, Ly, Lz of the periodic cell (nm); doubled cell: the doubled Lz; slab: the lengthened Lz */
  int geometry;         /* CPM_FINITE_FIELD, CPM_DOUBLED_CELL or CPM_SLAB */
  int kspace;           /* CPM_KSPACE_EWALD or CPM_KSPACE_PPPM */
  int precision;        /* CPM_FP64 or CPM_MIXED */
  double eta;           /* Gaussian width of electrode charges (Eq. 2), 1/nm */
  double alpha;         /* Ewald splitting of the per-step sums, 1/nm; alpha < eta/sqrt(2) */
  double rcut;          /* real-space cutoff of the per-step sums, nm */
  double kcut;          /* EWALD: k-sphere radius, 1/nm (all k != 0 with |k| <= kcut) */
  int mesh[3];          /* PPPM: mesh points per axis (each a product of 2, 3, 5) */
  int order;            /* PPPM: B-spline assignment order, 2..7 */
  /* converged Ewald parameters used once for the elastance matrix A */
  double alpha_build, rcut_build, kcut_build;
  int n_elec;           /* number of constant-potential electrode atoms */
  const double* elec_xyz;        /* host [3][n_elec] */
  const signed char* elec_side;  /* host [n_elec]: +1 positive, -1 negative electrode (d = side/2) */
  const unsigned char* elec_sub; /* host [n_elec]: doubled cell, 1 = first sub-cell (e1); NULL for finite field */
  int n_site;           /* number of electrolyte point charges */
  const double* site_q; /* host [n_site] charges (e); must sum to zero within 1e-9 */
  int flags;            /* CPM_FLAG_* bits, 0 for none */
} cpm_desc;

/* descriptor flags */
enum {
  /* capture each solve in a HIP graph on first use (per set of pointer
   * arguments and dv, 16 kept) and replay it afterwards; needs a non-null
   * stream.  Without it every call launches its kernels directly, which is
   * also what a caller capturing its own graph around the call needs. */
  CPM_FLAG_GRAPH = 1
};

/* Create a context: validates the descriptor (alpha < eta/sqrt2, positive
 * box and cutoffs, mesh factorable and its planes within LDS, neutral
 * electrolyte, sides +-1, doubled cell needs elec_sub with both sub-cells
 * non-empty, finite-field electrodes may not cross z = 0, slab electrodes
 * within half of the z period; all before any device call), uploads the
 * electrodes and prepares the per-step tables (k-vectors or influence
 * function, electrode spline weights, FFT twiddles, cell lists).
 * hip_stream may be NULL (the null stream).  *out is NULL on error. */
int cpm_create(const cpm_desc* desc, void* hip_stream, cpm_ctx** out);

/* Change the stream later calls enqueue on. */
int cpm_set_stream(cpm_ctx* ctx, void* hip_stream);

/* Once per electrode geometry (Eq. 3, 8-9, 14-15; "precomputed" in
 * Sec. II.A): builds A in FP64 (Gaussian real-space pairs, k-space as
 * 2 C C^T with C the sqrt(w)-weighted cos/sin factors, self term, and in
 * slab geometry the dipole correction's k_e 4 pi / V z z^T), inverts
 * it, projects S = O A^-1 (and O1 for the doubled cell) and forms S c.
 * Synchronises the stream.  CPM_ENOTSPD if A is not positive definite. */
int cpm_build_elastance(cpm_ctx* ctx);

/* One step of the path for one configuration: cell binning, real-space b,
 * k-space b (Ewald or PPPM), q* = S b + dV S c, k-space and real-space
 * forces on the sites (plus -Q_j dV/Lz along z for the finite field) and
 * the energies.
 *   site_xyz    device [3][n_site]
 *   dv          potential difference (V)
 *   q_out       device [n_elec]           electrode charges q*
 *   f_out       device [3][n_site] or NULL  forces on the sites (eV/nm)
 *   energy_out  device [2] or NULL          {U_coul, E_cp} (eV): U_coul =
 *               U_elyt - q.b + 1/2 q.A q; E_cp = U_coul - dV d.q
 *               (+ dV/Lz (z.q + sum Q_j Z_j) for the finite field; the slab
 *               correction is part of U_elyt, b and A), whose
 *               negative position gradient is f_out.
 * With CPM_FLAG_GRAPH, repeated calls with identical pointer arguments and
 * dv replay a HIP graph of the step.  CPM_ESTATE before
 * cpm_build_elastance. */
int cpm_solve(cpm_ctx* ctx, const double* site_xyz, double dv,
              double* q_out, double* f_out, double* energy_out);

/* Many frames and potential differences at once (frames independent):
 *   site_xyz   device [n_frames][3][n_site]
 *   dv_host    host [n_dv]
 *   q_out      device [n_frames][n_dv][n_elec]
 *   f_out      device [n_frames][n_dv][3][n_site] or NULL
 *   energy_out device [n_frames][n_dv][2] or NULL
 * The charges of all frames come from one GEMM Q = S B; q and the forces
 * are affine in dV, so each frame is solved once and the dV sweep is a
 * rank-one update.  Frames go through in launches of up to 4096: the first
 * call with at least 128 frames times launches of 64, 128, ... frames on its
 * own first frames and keeps the fastest size for the context, then at that
 * size times the site-pair tiles with 1, 2 and 4 workgroups per cell and the
 * x-y passes with one plane or as many as fit per workgroup, and keeps the
 * fastest of each (it synchronises the stream; setting CPM_BATCH_CHUNK in the
 * environment fixes the size and skips all of it).  CPM_ENOMEM if the
 * scratch does not fit. */
int cpm_solve_batch(cpm_ctx* ctx, int n_frames, const double* site_xyz,
                    int n_dv, const double* dv_host,
                    double* q_out, double* f_out, double* energy_out);

/* Fix the batch launch shapes instead of tuning them (for callers that tune
 * themselves, and for tests): frames per launch (1..4096), site-pair tile
 * workgroups per cell (1..64) and x-y planes per many-frame workgroup (0: as
 * many as fit in LDS, 1: one).  CPM_EINVAL outside those ranges. */
int cpm_set_batch_shape(cpm_ctx* ctx, int frames_per_launch, int tiles_per_cell, int xy_planes);

/* Gradient of L = sum_i (q*_i - t_i)^2 + U_coul(R, q*(R)) by the adjoint:
 * lambda = S [2 (q* - t) + dV c]; dL/dR_j is minus the Coulomb force on
 * site j with electrode charges q* - lambda; dL/ddV = lambda . c.
 *   q_target  device [n_elec]
 *   loss_out  device [1]; dl_dxyz device [3][n_site]; dl_ddv device [1]
 *   q_out     device [n_elec] or NULL (q* of the forward pass) */
int cpm_grad(cpm_ctx* ctx, const double* site_xyz, double dv, const double* q_target,
             double* loss_out, double* dl_dxyz, double* dl_ddv, double* q_out);

/* Laterally averaged charge density and electrostatic potential profile
 * across the cell (Eq. 16; potential-profile subsection and post-analysis
 * paragraph of the appendix), averaged over frames.  Grid: n_bins bins of
 * width h = Lz/n_bins, bin k = [k h, (k+1) h), values at the bin centres.
 * rho: the sites' point charges counted in the bin of their wrapped z, each
 * electrode atom's charge spread as its Gaussian (Eq. 2) integrated over
 * the bins (nearest periodic images included), divided by Lx Ly h and by
 * n_frames.  psi: the second-difference equations
 * (psi_{k+1} - 2 psi_k + psi_{k-1}) / h^2 = -rho_k / eps0 with, per geometry,
 * a rise of dv over one period (finite field), continuity (doubled cell) or
 * zero field at z = 0 (slab), solved exactly; the mean of psi over the bins
 * centred in [bulk_lo, bulk_hi) is subtracted.
 *   site_xyz  device [n_frames][3][n_site]
 *   q         device, frame f's electrode charges at q + f * q_stride
 *             (q_stride >= n_elec; n_dv * n_elec to read one dV of a batch)
 *   rho_out   device [n_bins] (e/nm^3); psi_out device [n_bins] (V)
 * CPM_EINVAL for n_bins outside 2..2048, an empty bulk window or more than
 * 2048 distinct electrode heights.  The scratch (n_part x (n_bins + heights)
 * doubles, n_part <= 128) is allocated by the context and grows on demand
 * (that call synchronises the stream). */
int cpm_profile(cpm_ctx* ctx, int n_frames, const double* site_xyz, const double* q, long long q_stride,
                double dv, int n_bins, double bulk_lo, double bulk_hi, double* rho_out, double* psi_out);

/* cpm_profile for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, results and errors, but the histogram scratch is a
 * file-scope device array of 4 MiB per GPU (128 partitions x (2048 bins +
 * 2048 heights) doubles, the most the argument limits allow; a request
 * beyond it is CPM_EINVAL) whose address the library resolves once per
 * device when a context is created, so the call itself allocates nothing
 * and never synchronises.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (on different streams, or from different
 * contexts) race.  Each partition is written whole before it is read, so no
 * clearing is needed between calls. */
int cpm_profile_noalloc(cpm_ctx* ctx, int n_frames, const double* site_xyz, const double* q, long long q_stride,
                        double dv, int n_bins, double bulk_lo, double bulk_hi, double* rho_out, double* psi_out);

/* ---------------------------------------------------------------- MD loop
 * The constant-potential MD loop of the paper's simulations (appendix,
 * force-field and production paragraphs): velocity Verlet, a Nose-Hoover
 * thermostat on the electrolyte (one per group; the doubled cell uses one
 * per sub-cell), rigid three-site molecules held by SHAKE and RATTLE,
 * Lennard-Jones site-site (different molecules) and site-graphene
 * interactions cut at lj_cut with the energy shifted to zero there
 * (Lorentz-Berthelot), and the Coulomb forces of this context with the
 * electrode charges re-solved every charge_every steps (between updates the
 * forces use the last charges).  Units: nm, ps, amu, kJ/mol.  Per step:
 *   thermostat half step; v += dt/2 F/m; x += dt v; SHAKE; v = dx/dt;
 *   F = F_LJ + F_Coulomb; v += dt/2 F/m; RATTLE; thermostat half step,
 * the thermostat half step being xi += dt/4 (K2 - N_f kT)/Q; eta += dt/2 xi;
 * v *= exp(-xi dt/2); xi += dt/4 (K2' - N_f kT)/Q with K2 = sum m v^2,
 * N_f = 3 sites - 3 per rigid molecule, Q = N_f kT tau^2. */
typedef struct cpm_md cpm_md;
typedef struct {
  int n_mol;                  /* molecules, in site order */
  const int* mol_size;        /* host [n_mol]: 3 (rigid: sides bond, bond, bond sqrt 3 from the first site) or 1 */
  const int* mol_group;       /* host [n_mol]: thermostat group, 0 .. n_groups-1 */
  int n_groups;               /* 1 or 2 */
  const double* site_mass;    /* host [n_site] amu */
  const double* site_sigma;   /* host [n_site] nm */
  const double* site_eps;     /* host [n_site] kJ/mol */
  int n_lj_elec;              /* graphene atoms taking part in the Lennard-Jones sums (fixed) */
  const double* lj_elec_xyz;  /* host [3][n_lj_elec] */
  double carbon_sigma, carbon_eps;
  double lj_cut;              /* nm, below half the smallest box length */
  double bond;                /* nm */
  double dt;                  /* ps */
  double temperature;         /* K */
  double tau;                 /* ps, thermostat time constant */
  int charge_every;           /* charge update every this many steps */
} cpm_md_desc;

/* MD loop on a built FP64 context (which it uses for the Coulomb forces and
 * must not be destroyed first).  Copies the tables; CPM_EINVAL for a bad
 * table, CPM_ESTATE before cpm_build_elastance. */
int cpm_md_create(cpm_ctx* ctx, const cpm_md_desc* desc, cpm_md** out);

/* n_steps steps from the state in x and v (device [3][n_site], updated in
 * place).  The first call makes v normal to the constraints and evaluates
 * the forces with a charge solve; later calls continue from the forces,
 * charges and thermostat state the loop holds (so x and v must be the last
 * call's).  q_out (device [n_elec] or NULL): the charges of the last update;
 * thermo_out (device [n_steps][4] or NULL): per step the kinetic energy, the
 * Lennard-Jones energy, E_cp of the last charge update and the thermostat's
 * energy sum_g (Q xi^2/2 + N_f kT eta) (kJ/mol).  Asynchronous.  Between
 * charge updates the steps reuse the electrode charge's mesh spectrum and
 * cell-sorted charges of the loop's last update (PPPM); any other call on
 * the context in between (a solve, replayed graph included, a batch,
 * another loop) makes the next step rebuild them from the loop's own
 * charges, so calls may be interleaved without changing the trajectory. */
int cpm_md_run(cpm_md* md, double* x, double* v, double dv, int n_steps, double* q_out, double* thermo_out);

/* Thermostat variables (host [n_groups] each, nullable) and the step count;
 * synchronises. */
int cpm_md_state(cpm_md* md, double* xi_host, double* eta_host, long long* step_host);

/* Switch the thermostat off (0: constant energy) or on (default). */
int cpm_md_set_thermostat(cpm_md* md, int on);

void cpm_md_destroy(cpm_md* md);

/* Copies of internal matrices for tests and checkpoints (synchronises):
 * which = 0: A, 1: S (projected inverse), 2: S c (n_elec values).
 * host_out holds n_elec*n_elec (or n_elec) doubles. */
int cpm_get_matrix(cpm_ctx* ctx, int which, double* host_out);

/* Restore S (and S c) from a host copy instead of building (checkpoint
 * resume); marks the context built.  host_S [n_elec][n_elec]. */
int cpm_set_matrix(cpm_ctx* ctx, const double* host_S);

/* Internal per-step buffers of the last cpm_solve, copied to the host
 * (synchronises).  Returns the element count, or a negative status.
 * host_out may be NULL to query the count.
 *   CPM_BUF_CELL_START int32 [n_cells+1]   CPM_BUF_SITE_ORDER int32 [n_site]
 *   CPM_BUF_PHI_REAL  double [n_elec]  real-space electrolyte potential at electrodes (V)
 *   CPM_BUF_B         double [n_elec]  the vector b
 *   CPM_BUF_RHO_MESH  double [Kz][Ky][Kx] electrolyte charge mesh
 *   CPM_BUF_PHI_MESH  double [Kz][Ky][Kx] electrolyte potential mesh (V)
 *   CPM_BUF_FIELD_MESH double [3][Kz][Ky][Kx] field of all charges (V/nm)
 *   CPM_BUF_NCELL     int32 [3]  cells per axis
 *   CPM_BUF_BATCH_CHUNK int32 [3] the batch tuner's choices: frames per launch (0: not tuned yet),
 *                       site-pair tile workgroups per cell, x-y planes per workgroup (0: as many as fit)
 * The meshes are those of a cpm_solve: cpm_solve_batch does not store the
 * charge mesh, transforms the potential only on the planes the electrode
 * stencils reach and, at spline order 5, interpolates the field at the sites
 * without storing its mesh. */
enum {
  CPM_BUF_CELL_START = 0, CPM_BUF_SITE_ORDER = 1, CPM_BUF_PHI_REAL = 2, CPM_BUF_B = 3,
  CPM_BUF_RHO_MESH = 4, CPM_BUF_PHI_MESH = 5, CPM_BUF_FIELD_MESH = 6, CPM_BUF_NCELL = 7,
  CPM_BUF_BATCH_CHUNK = 8
};
long long cpm_get_buffer(cpm_ctx* ctx, int which, void* host_out);

/* Kernels of the step, for timing.  cpm_replay_kernel re-enqueues the most
 * recent launch of one of them `reps` times with the same arguments on the
 * context's stream (callers bracket it with events to time one kernel).  It
 * overwrites internal buffers only; outputs of the last step stay valid.
 * CPM_ESTATE if that kernel has not run yet. */
enum {
  CPM_KERNEL_BIN = 0, CPM_KERNEL_REAL_B, CPM_KERNEL_SITE_PAIRS, CPM_KERNEL_FFT_XY_FWD,
  CPM_KERNEL_FFT_Z_POT, CPM_KERNEL_FFT_XY_INV, CPM_KERNEL_GATHER_B, CPM_KERNEL_CHARGES,
  CPM_KERNEL_SPREAD_ELEC, CPM_KERNEL_FFT_XY_FWD_E, CPM_KERNEL_FFT_Z_FIELD, CPM_KERNEL_FFT_XY_INV_E,
  CPM_KERNEL_SITE_FORCES, CPM_KERNEL_ENERGY,
  /* batched form only: the charge GEMM Q0 = S B (FP64, or the bf16 split
   * products in MIXED), the expansion of q over the dV sweep, and that of
   * the forces */
  CPM_KERNEL_GEMM, CPM_KERNEL_EXPAND_Q, CPM_KERNEL_EXPAND_F,
  CPM_KERNEL_COUNT
};
int cpm_replay_kernel(cpm_ctx* ctx, int kernel, int reps);

/* Synchronise the stream and report errors raised inside kernels since the
 * last call (CPM_ENONFINITE for non-finite positions), then clear them. */
int cpm_sync_status(cpm_ctx* ctx);

/* Message of the last error on this context (or of the last failed
 * cpm_create when ctx is NULL).  Never NULL. */
const char* cpm_last_error(const cpm_ctx* ctx);

/* Free every device allocation and graph of the context.  NULL is a no-op. */
void cpm_destroy(cpm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* CPM_H */
