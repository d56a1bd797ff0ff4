/*
 * tlb.h - C ABI of libtlb, an MI355X (gfx950) implementation of the ternary
 * free-energy lattice Boltzmann method of Semprebon, Krueger & Kusumaatmaja
 * (arXiv:1511.02155).
 *
 * What one time step computes (Sec. IV of the paper):
 *   - moments rho = sum f, rho v = sum f e, phi = sum g, psi = sum k (eq. lbconstraint);
 *   - concentrations C1 = (rho+phi-psi)/2, C2 = (rho-phi-psi)/2, C3 = psi (Sec. II.C);
 *   - gradients and Laplacians of C_m with isotropic lattice stencils, using
 *     ghost rows at walls that impose alpha^2 kappa_m grad_perp C_m = -h_m
 *     (Sec. II.B, eq. cahn_gradient);
 *   - chemical potentials mu_phi, mu_psi and the pressure-tensor terms (Sec. III);
 *   - equilibria f^eq, g^eq, k^eq (eq. eqdistfbinary), BGK collision with
 *     tau_f, tau_g (= tau_phi), tau_k (= tau_psi) (eq. latboltCollision);
 *   - propagation (eq. latboltPropagation) with half-way bounce-back at walls.
 *
 * Lattices and layouts
 *   D2Q9 velocities, index order: 0 (0,0); 1 (1,0); 2 (-1,0); 3 (0,1); 4 (0,-1);
 *     5 (1,1); 6 (1,-1); 7 (-1,1); 8 (-1,-1).
 *   D3Q19 velocities, index order (the order of the weight index sets printed in
 *     Sec. IV): 0 rest; 1,2 = +-x; 3,4 = +-y; 5,6 = +-z; 7..10 = (1,1,0),
 *     (1,-1,0), (-1,1,0), (-1,-1,0); 11..14 = (0,1,1), (0,1,-1), (0,-1,1),
 *     (0,-1,-1); 15..18 = (1,0,1), (1,0,-1), (-1,0,1), (-1,0,-1).
 *   Node index n = x + nx*(y + ny*z), N = nx*ny*nz.  x and z are periodic; y is
 *   periodic or bounded by two half-way walls (below y = 0 and above y = ny-1).
 *   Concentrations / fields: [component][N].  Velocities: [D][N].
 *   Populations of one species: [Q][N].  Species 0 = f, 1 = g, 2 = k.
 *   Wetting parameters of one wall: [component m = 0..2][x + nx*z].
 *
 * Ownership and threading
 *   A tlb_sim owns all of its device memory.  Host arrays passed in are
 *   borrowed for the duration of the call.  Host-I/O calls (plain names) are
 *   ordered on the simulation's stream and return after the data has been
 *   copied.  *_dev calls take device pointers in the simulation's own precision
 *   (float for TLB_F32, double for TLB_F64), are enqueued on the simulation's
 *   stream and do not synchronise.  A tlb_sim must not be used from two host
 *   threads at once.
 *
 * Errors
 *   Every call returns a tlb_status: TLB_OK (0) or a negative code.
 *   TLB_EINVAL  invalid argument (parameters outside the ranges below, NULL
 *               pointer, index out of range);
 *   TLB_ENOMEM  device allocation failed;
 *   TLB_EHIP    a HIP runtime call failed (tlb_last_hip_error() gives the code);
 *   TLB_ENAN    a non-finite population was detected;
 *   TLB_ESTATE  call out of order (e.g. tlb_step before any initialisation).
 */
#ifndef TLB_H
#define TLB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TLB_OK = 0,
    TLB_EINVAL = -1,
    TLB_ENOMEM = -2,
    TLB_EHIP = -3,
    TLB_ENAN = -4,
    TLB_ESTATE = -5
} tlb_status;

enum { TLB_D2Q9 = 0, TLB_D3Q19 = 1 };
enum { TLB_F32 = 0, TLB_F64 = 1 };
enum { TLB_BGK = 0, TLB_MRT = 1 };
/* Largest number of fluid components (tlb_params.ncomp). */
enum { TLB_MAX_COMP = 5 };

/* Field selectors of tlb_get_field. */
enum {
    TLB_FIELD_C1 = 0,
    TLB_FIELD_C2 = 1,
    TLB_FIELD_C3 = 2,
    TLB_FIELD_RHO = 3,
    TLB_FIELD_PHI = 4,
    TLB_FIELD_PSI = 5,
    TLB_FIELD_UX = 6,
    TLB_FIELD_UY = 7,
    TLB_FIELD_UZ = 8,
    TLB_FIELD_MU_PHI = 9,
    TLB_FIELD_MU_PSI = 10,  /* mu of psi_3 = C3 */
    TLB_NFIELDS = 11,       /* the selectors of a three-component simulation */
    TLB_FIELD_C4 = 11,      /* C4, C5: simulations with ncomp >= 4, 5 */
    TLB_FIELD_C5 = 12
};

/*
 * Simulation parameters.
 *   lattice   TLB_D2Q9 (requires nz == 1) or TLB_D3Q19 (requires nz >= 3).
 *   prec      TLB_F32 or TLB_F64: storage precision of the populations.  D2Q9
 *             computes in FP64 for both (FP32 storage then rounds each population
 *             once per step); D3Q19 computes in the storage precision.
 *   nx, ny    lattice size, each >= 3; nz >= 1.
 *   walls_y   0: periodic in y; 1: half-way walls below y = 0 and above y = ny-1.
 *   kappa[m]  bulk coefficients kappa_1..3 > 0 (Sec. II.A); kappa'_m = alpha^2 kappa_m.
 *   alpha     interface width parameter > 0 (Sec. II.A).
 *   tau_f, tau_g, tau_k   relaxation times of f, g, k, each > 1/2 (Sec. IV).
 *   gamma_phi, gamma_psi  the tunable Gamma_phi, Gamma_psi of the g and k
 *             equilibria; mobilities are M = Gamma (tau - 1/2) (Sec. IV).
 *   no_advection  0: the g and k equilibria carry the fluid velocity (advective
 *             Cahn-Hilliard equations, Sec. III); 1: their velocity terms are left
 *             out, which removes advection from the Cahn-Hilliard equations (the
 *             diffusive coarsening runs of Sec. V.C).  Zero-initialised
 *             parameters keep the advective model.
 *   collision TLB_BGK (single relaxation time, eq. latboltCollision) or
 *             TLB_MRT: f relaxes with multiple relaxation times, the
 *             extension Sec. IV names, f* = f - M^-1 S M (f - f^eq) in the
 *             orthogonal polynomial moment basis of the lattice (Lallemand &
 *             Luo for D2Q9, d'Humieres et al. for D3Q19); the viscous stress
 *             moments relax at 1/tau_f (shear viscosity (tau_f - 1/2)/3), the
 *             energy moment at 1/tau_bulk (bulk viscosity
 *             (2/D)(tau_bulk - 1/2)/3) and all other moments at 1/tau_ghost.
 *             g and k always relax with BGK.  With tau_bulk = tau_ghost =
 *             tau_f, MRT is BGK.  The batched step and the reverse step take
 *             BGK only (TLB_EINVAL otherwise).
 *   tau_bulk, tau_ghost  MRT relaxation times, each > 1/2 (ignored for BGK).
 *   ncomp     number of fluid components N, 3 .. TLB_MAX_COMP (0 means 3).
 *             N > 3 (Sec. II.E, both lattices) uses rho = sum_m C_m, phi = C1 - C2
 *             and psi_l = C_l for l >= 3, with one k population set per psi_l
 *             (species 2 .. N-1, all relaxing with tau_k and using gamma_psi)
 *             and mu_psi_l = mu_l - (mu_1 + mu_2)/2.  Every per-component
 *             array then has N rows: kappa_m (kappa[0..2] and kappa_hi[0..N-4]),
 *             the wetting parameters [N][nx*nz], the initial fields C[N][..]
 *             and the populations [N][Q][..].  The batched step and the reverse
 *             step take three components only.
 *   kappa_hi  kappa_4 .. kappa_N, each > 0 (ignored for N = 3).
 */
typedef struct {
    int32_t lattice;
    int32_t prec;
    int32_t nx, ny, nz;
    int32_t walls_y;
    double kappa[3];
    double alpha;
    double tau_f, tau_g, tau_k;
    double gamma_phi, gamma_psi;
    int32_t no_advection;
    int32_t collision;
    double tau_bulk, tau_ghost;
    int32_t ncomp;
    double kappa_hi[TLB_MAX_COMP - 3];
} tlb_params;

/* Conservation and stability check of the current state s_t (all sums in FP64). */
typedef struct {
    double mass[3];     /* sum rho, sum phi, sum psi over fluid nodes */
    double momentum[3]; /* sum rho v */
    double max_speed;   /* max |v| */
    int64_t nonfinite;  /* number of nodes with a non-finite moment */
    int64_t step;       /* time steps taken since initialisation */
    /* sum over fluid nodes of C_m^2 (1 - C_m)^2.  A flat interface of the profile of eq. (tanh)
     * contributes alpha/6 per unit length (area in 3D), so 6 * interface[m] / alpha estimates the
     * length (area) of the boundary of component m and chi_m of Sec. V.C is its value divided by
     * the side of a square domain; the typical domain size is the domain area over that length. */
    double interface[3];
    /* N > 3: sum psi_l and the interface sums of C_l for l = 4 .. N (zero beyond N) */
    double mass_hi[TLB_MAX_COMP - 3];
    double interface_hi[TLB_MAX_COMP - 3];
} tlb_diag;

typedef struct tlb_sim tlb_sim;

/* Text of a status code (static storage). */
const char* tlb_status_str(int status);
/* HIP error code of the last TLB_EHIP returned on this thread (0 if none). */
int tlb_last_hip_error(void);
/* ABI version (major * 100 + minor); 2xx: tlb_params.no_advection and tlb_diag.interface;
 * 3xx: tlb_params.collision, tau_bulk, tau_ghost; 4xx: tlb_params.ncomp, kappa_hi and
 * tlb_diag.mass_hi, interface_hi (N components); 5xx: tlb_adjoint_step (in place) and the
 * wetting range counts. */
int tlb_version(void);

/*
 * Create a simulation on the current HIP device.  stream: a hipStream_t to
 * enqueue all work on, or NULL to let the simulation create (and own) one.
 * The state is undefined until tlb_init_equilibrium or tlb_set_populations.
 * Wetting parameters start at zero (neutral walls).
 * TLB_EINVAL for parameters outside the ranges documented with tlb_params, and
 * for lattices beyond the 32-bit offsets of the buffer instructions: each
 * descriptor covers at most 4 GiB - 256 bytes, which is one population array
 * on D2Q9 (nx * ny * sizeof) and one z plane of all populations on D3Q19
 * (ceil(nx * ny / 64) * 64 * 19 * N * sizeof).  TLB_ENOMEM when the two state
 * buffers do not fit on the device.
 */
tlb_status tlb_create(const tlb_params* params, void* stream, tlb_sim** out);
tlb_status tlb_destroy(tlb_sim* sim);
tlb_status tlb_get_params(const tlb_sim* sim, tlb_params* out);

/*
 * Wetting parameters h_m of one wall (Sec. II.B, eq. Cahn): wall 0 = below
 * y = 0, wall 1 = above y = ny-1; h: host array [N][nx*nz] (N components,
 * 3 unless tlb_params.ncomp says more), finite values (TLB_EINVAL otherwise).
 * Requires walls_y == 1.  Takes effect from the next step (or initialisation).
 * Values with |4 h_m / (alpha kappa_m)| > 1 lie outside the range in which the
 * surface free energy of Sec. II.B gives closed-form wall concentrations and
 * contact angles; they are accepted and applied as given (the ghost-row
 * condition alpha^2 kappa_m d_perp C_m = -h_m does not need that range), the
 * first such call of a simulation prints one warning line to stderr, and
 * tlb_wetting_outside_range reports how many values of both walls are outside
 * it (-1 if a wall was last set through tlb_set_wetting_dev, whose device
 * values are not inspected).  tlb_set_kappa recounts.
 */
tlb_status tlb_set_wetting(tlb_sim* sim, int wall, const double* h);
tlb_status tlb_wetting_outside_range(const tlb_sim* sim, int64_t* count);

/*
 * Initialise s_0 to the equilibria of the concentration fields C (host,
 * [ncomp][N], rho = sum_m C_m, phi = C1 - C2, psi_l = C_l, Sec. II.C, II.E) and the
 * velocity u (host, [D][N]; NULL = at rest), with the gradient terms of the
 * equilibria evaluated from C.  Resets the step counter.
 */
tlb_status tlb_init_equilibrium(tlb_sim* sim, const double* C, const double* u);

/* Advance the state by nsteps >= 0 time steps (asynchronous on the stream).
 * One time step is the lattice Boltzmann update of Sec. IV: collision of f, g
 * and k towards their equilibria (eq. latboltCollision, with the equilibria of
 * eq. eqdistfbinary built from the chemical potentials and pressure tensor of
 * Sec. III and the wetting condition of Sec. II.B) followed by propagation
 * (eq. latboltPropagation) with half-way bounce-back at the walls.
 * TLB_EINVAL for nsteps < 0, TLB_ESTATE before the state is initialised,
 * TLB_ENAN from the periodic check of tlb_set_check_every. */
tlb_status tlb_step(tlb_sim* sim, int64_t nsteps);

/*
 * Check for non-finite populations every `every` steps inside tlb_step
 * (0 = never, the default).  A check synchronises the stream; tlb_step then
 * returns TLB_ENAN when one is found.
 */
tlb_status tlb_set_check_every(tlb_sim* sim, int64_t every);

/*
 * Replay the steps of tlb_step from a captured hipGraph in chains of
 * steps_per_graph launches (an even number; 0, the default, launches every step
 * directly).  For small lattices, where a step takes about as long as its
 * launch, this removes most of the launch overhead.  The chain is captured on
 * the simulation's stream at the first tlb_step that needs it and replayed
 * after that; tlb_set_launch and tlb_set_kappa drop it (the launches hold the
 * shape and the coefficients), wetting parameters and states are read from
 * device memory and need no new capture.  Results are bit for bit those of
 * direct launches.  The capture must not overlap other work enqueued on the
 * same stream from another thread.  TLB_EINVAL for an odd or negative count.
 */
tlb_status tlb_set_graph(tlb_sim* sim, int64_t steps_per_graph);

/* Macroscopic field `which` (TLB_FIELD_*) of the state s_t into host out[N]
 * (TLB_EINVAL for an unknown selector, TLB_ESTATE before initialisation).
 * rho, phi, psi and rho v are the moments of eq. lbconstraint (Sec. IV),
 * v = (rho v) / rho; C1 = (rho + phi - psi)/2, C2 = (rho - phi - psi)/2,
 * C3 = psi (Sec. II.C; C_l = psi_l for N > 3, Sec. II.E); mu_phi and mu_psi are
 * the chemical potentials of Sec. III with the gradients of the step. */
tlb_status tlb_get_field(tlb_sim* sim, int which, double* out);

/* Post-propagation populations s_t of one species (0 f, 1 g, 2 .. ncomp-1 the
 * k sets of psi_3 ..) into host out[Q][N]: the distributions of eq.
 * latboltPropagation after the last step (TLB_EINVAL for an unknown species). */
tlb_status tlb_get_populations(tlb_sim* sim, int species, double* out);

/* Overwrite the populations s_t of one species from host in[Q][N]. */
tlb_status tlb_set_populations(tlb_sim* sim, int species, const double* in);

/* Mass, momentum, max |v| and a non-finite count of s_t, from the moments of
 * eq. lbconstraint (Sec. IV): sum rho, sum phi and sum psi are conserved by the
 * collision and by propagation with bounce-back, and sum rho v on fully periodic
 * lattices; max |v| is the spurious-velocity measure of the equilibria of Sec.
 * V.A.  Sums run over the fluid nodes in a fixed order (reproducible).  Returns
 * TLB_ENAN (with *out filled) when non-finite values are present. */
tlb_status tlb_diagnostics(tlb_sim* sim, tlb_diag* out);

/* Time steps taken since initialisation. */
tlb_status tlb_get_step(const tlb_sim* sim, int64_t* step);

/* Wait for all work enqueued by this simulation. */
tlb_status tlb_synchronize(tlb_sim* sim);

/* The hipStream_t this simulation enqueues on. */
void* tlb_get_stream(const tlb_sim* sim);

/*
 * Checkpoint and resume.  The raw state is the stored population buffer of
 * the current step in the simulation's own representation (tlb_state_bytes()
 * bytes); saving and loading it resumes a run bit for bit.  tlb_save_state /
 * tlb_load_state copy to / from host memory and synchronise;  the _dev forms
 * copy to / from device memory asynchronously.  Loading keeps the step count
 * given by `step`.
 */
int64_t tlb_state_bytes(const tlb_sim* sim);
tlb_status tlb_save_state(tlb_sim* sim, void* host_dst, int64_t* step);
tlb_status tlb_load_state(tlb_sim* sim, const void* host_src, int64_t step);
tlb_status tlb_save_state_dev(tlb_sim* sim, void* dev_dst);
tlb_status tlb_load_state_dev(tlb_sim* sim, const void* dev_src, int64_t step);

/*
 * Change kappa_1..N (kappa[ncomp], each > 0) between runs; the wetting ghost
 * values h_m / (alpha^2 kappa_m) are recomputed from the h_m last set.
 */
tlb_status tlb_set_kappa(tlb_sim* sim, const double* kappa);

/* ------------------------------------------------------------------------ */
/* Contact angles and wetting parameters (host-only helpers; no GPU use)    */
/* ------------------------------------------------------------------------ */
/*
 * Young's law cos(theta_mn) = (gamma_sn - gamma_sm) / gamma_mn with the
 * fluid-fluid tensions gamma_mn = alpha (kappa_m + kappa_n) / 6 (Sec. II.A)
 * and the solid-fluid tensions of the surface free energy (Sec. II.B, eq.
 * solidST) reduces to
 *   cos(theta_mn) = (Phi_m - Phi_n) / (2 (kappa_m + kappa_n)),
 *   Phi_m = kappa_m (s+^3 - s-^3),  s+- = sqrt(1 +- 4 h_m / (alpha kappa_m)).
 * (The inversion formula printed in Sec. II.D has the opposite sign and an
 * extra factor alpha; these helpers use the relation above.)  Angles are in
 * degrees, theta_mn measured through fluid m; kappa[3] > 0, alpha > 0.
 *
 * tlb_contact_angles: theta_out = (theta_12, theta_23, theta_31) for h[3]
 *   with |4 h_m / (alpha kappa_m)| <= 1 (TLB_EINVAL otherwise).
 * tlb_wetting_from_angles: h_out[3] that gives theta_12 and theta_23 (theta_31
 *   follows from the Girifalco-Good relation) with the redundancy condition
 *   sum_m h_m / kappa_m = 0 of Sec. II.D (zero density gradient at the wall);
 *   TLB_EINVAL if no such h exists within |4 h_m / (alpha kappa_m)| <= 1.
 */
tlb_status tlb_contact_angles(const double* kappa, double alpha, const double* h, double* theta_out);
tlb_status tlb_wetting_from_angles(const double* kappa, double alpha, double theta12, double theta23,
                                   double* h_out);

/* ------------------------------------------------------------------------ */
/* Reverse mode (D2Q9; TLB_EINVAL for D3Q19)                                 */
/* ------------------------------------------------------------------------ */
/*
 * Adjoint variables lambda live in the layout of the raw state
 * (tlb_state_bytes() bytes, native precision): lambda_t = dL/du_t where u_t
 * is the stored state of step t.  One reverse step maps lambda_{t+1} to
 *   lambda_t = (d u_{t+1} / d u_t)^T lambda_{t+1}
 * and adds (d u_{t+1} / d theta)^T lambda_{t+1} to the gradients of
 * theta = (h_m of both walls, kappa_m) (the initial state is held fixed).
 *
 * tlb_adjoint_seed_dev: lambda_T from dL/dC of the final state s_T;
 *   dLdC_dev: [3][N] native precision (dL/dC1, dL/dC2, dL/dC3) or NULL (zero).
 * tlb_adjoint_step_dev: one reverse step; state_dev is the raw state u_t
 *   (from tlb_save_state_dev or a checkpoint); lambda_in_dev != lambda_out_dev;
 *   dh_dev [2][3][nx] FP64 and dkappa_dev [3] FP64 are accumulated into
 *   (either may be NULL).
 * tlb_forward_checkpointed: advance nsteps from the current state, storing the
 *   raw state before steps 0, every, 2*every, ... into ckpt_dev, which holds
 *   tlb_checkpoint_slots(nsteps, every) states (every ~ sqrt(nsteps)).
 * tlb_adjoint_backward: with those checkpoints, run the whole reverse pass
 *   for dL/dC of the state after nsteps: each segment is recomputed from its
 *   checkpoint into internal scratch and traversed backwards.  The scratch is
 *   two buffers of `every` states: the recompute of the next segment runs on a
 *   stream of the library's own (default priority) while the current segment
 *   is reversed on the simulation's stream, which waits for it before the
 *   call's work ends.  The simulation's own state is not changed.
 */
/*
 * tlb_adjoint_step: the in-place form of tlb_adjoint_step_dev.  lambda_dev
 *   holds lambda_{t+1} on entry and lambda_t on return; dh_dev is
 *   [2][3][nx*nz] FP64 (nz = 1), dkappa_dev [3] FP64, both accumulated (either
 *   may be NULL).  It runs the same kernel into an internal buffer and copies
 *   the result back, so it moves one more state than the out-of-place form.
 *   The first reverse-mode call of a simulation allocates its adjoint buffers.
 */
tlb_status tlb_adjoint_seed_dev(tlb_sim* sim, const void* dLdC_dev, void* lambda_dev);
tlb_status tlb_adjoint_step(tlb_sim* sim, const void* state_dev, void* lambda_dev, double* dh_dev,
                            double* dkappa_dev);
tlb_status tlb_adjoint_step_dev(tlb_sim* sim, const void* state_dev, const void* lambda_in_dev,
                                void* lambda_out_dev, double* dh_dev, double* dkappa_dev);
/*
 * tlb_adjoint_step_noalloc: tlb_adjoint_step_dev for callers that cannot
 *   allocate device memory during the call (code under HIP graph capture,
 *   tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 *   kernels, launch shape and results (bit for bit) as tlb_adjoint_step_dev,
 *   but the call allocates nothing: its scratch (the per-work-item dL/dkappa
 *   partials, which the call writes before it reduces them, and, when dh_dev is
 *   NULL, a sink for dL/dh, which it clears) lives in a static device array of
 *   TLB_NOALLOC_SCRATCH_BYTES per GPU, which each GPU the library runs on holds
 *   until the process ends.  A simulation needs
 *   tlb_adjoint_step_noalloc_scratch(sim) bytes of it
 *   (3 * work items + 6 * nx * nz doubles); larger ones return
 *   TLB_EINVAL.  Every call on one GPU uses that GPU's single array: calls that
 *   overlap on one GPU (other streams, other host threads) race and must be
 *   serialised by the caller.  The first call on a device looks up the array's
 *   address (no allocation); it may be made before any capture starts.
 */
#define TLB_NOALLOC_SCRATCH_BYTES (1 << 20)
tlb_status tlb_adjoint_step_noalloc(tlb_sim* sim, const void* state_dev, const void* lambda_in_dev,
                                    void* lambda_out_dev, double* dh_dev, double* dkappa_dev);
int64_t tlb_adjoint_step_noalloc_scratch(const tlb_sim* sim);
int64_t tlb_checkpoint_slots(int64_t nsteps, int64_t every);
tlb_status tlb_forward_checkpointed(tlb_sim* sim, int64_t nsteps, int64_t every, void* ckpt_dev);
tlb_status tlb_adjoint_backward(tlb_sim* sim, int64_t nsteps, int64_t every, const void* ckpt_dev,
                                const void* dLdC_dev, double* dh_dev, double* dkappa_dev);

/* Device-pointer variants (native precision, asynchronous). */
tlb_status tlb_init_equilibrium_dev(tlb_sim* sim, const void* C_dev, const void* u_dev);
tlb_status tlb_get_field_dev(tlb_sim* sim, int which, void* out_dev);
tlb_status tlb_get_populations_dev(tlb_sim* sim, int species, void* out_dev);
tlb_status tlb_set_populations_dev(tlb_sim* sim, int species, const void* in_dev);
tlb_status tlb_set_wetting_dev(tlb_sim* sim, int wall, const void* h_dev);

/*
 * Launch shape of the fused step kernel.
 *   D2Q9: each workgroup sweeps a strip of `width` columns (64, 128 or 256)
 *     over `chunk` rows; variant 1 prefetches the next row's populations while
 *     the current row is collided, variant 0 does not.
 *   D3Q19: each workgroup sweeps a tile of width x height columns (32x8 or
 *     64x4) over `chunk` planes; variant 1 keeps the next plane's populations in registers
 *     between their two uses, variant 0 reads them a second time from cache;
 *     variant 2 (FP32 storage, three or four components) also issues the loads of the plane
 *     after next before the current plane is collided.
 *   chunk >= 1; chunk = 0 picks a default.  The default shape depends on the
 *   lattice size and precision.  For a given variant, results are bitwise
 *   identical for every shape.  The D2Q9 variants are bitwise identical to each
 *   other; the D3Q19 variants are separate kernels whose results agree to
 *   rounding (the compiler may fuse different multiply-adds).  An invalid shape
 *   returns TLB_EINVAL.
 */
typedef struct {
    int32_t width, height, chunk, variant;
} tlb_launch;
tlb_status tlb_set_launch(tlb_sim* sim, const tlb_launch* launch);
tlb_status tlb_get_launch(const tlb_sim* sim, tlb_launch* out);

/* Launch shape of the reverse step (D2Q9 only; TLB_EINVAL otherwise).  A
 * workgroup holds `height` row groups (1, 2 or 4; 0 means 1) of `width` lanes
 * (64, 128 or 256; width * height <= 256).  It covers `width` columns,
 * produces the middle width - 6 of them, and sweeps `chunk` rows (chunk >= 1;
 * 0 picks a default), height rows per iteration.  Variant 0 issues the loads
 * of stage 4 (the gather of lambda_{t+1}) when that stage starts; variant 1
 * issues the loads of all four stages of a row before its arithmetic;
 * variant 2 is variant 0 that also loads the next iteration's pull and
 * lambda_{t+1} rows during the current one.  For a given variant the adjoint
 * populations and dL/dh are bitwise the same for every shape; the variants
 * fuse multiply-adds differently and agree to rounding.  dL/dkappa is summed
 * per work item, so its last bits depend on the shape (it is reproducible for
 * a fixed shape). */
tlb_status tlb_set_adjoint_launch(tlb_sim* sim, const tlb_launch* launch);
tlb_status tlb_get_adjoint_launch(const tlb_sim* sim, tlb_launch* out);

/* Algorithmic HBM bytes one fused step moves per fluid node (read + write). */
double tlb_bytes_per_node(const tlb_sim* sim);

/*
 * Propagation alone: nsteps >= 0 times the pull of the fused step (with
 * half-way bounce-back, eq. latboltPropagation) and its store, with no
 * collision, in the step's work decomposition and current launch shape (the
 * D3Q19 tiles without their ring).  It moves exactly the bytes of a step in
 * exactly its access pattern, so its bandwidth is the ceiling that pattern
 * leaves the fused step.  It changes the state (to the free-streamed one) but
 * not the step counter; a measurement call.  Asynchronous on the stream.
 */
tlb_status tlb_stream_only(tlb_sim* sim, int64_t nsteps);

/*
 * Plain device-to-device copy kernel (16-byte vector loads and stores) of
 * `bytes` bytes (a multiple of 16; both pointers 16-byte aligned), enqueued
 * on `stream` (NULL: the null stream).  It is the bandwidth reference the
 * step kernels are measured against: its runtime gives the attainable copy
 * bandwidth and its hardware byte counters calibrate the step kernels'.
 */
tlb_status tlb_device_copy(void* dst, const void* src, int64_t bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Batched D2Q9 lattices                                                    */
/* ------------------------------------------------------------------------ */
/*
 * A batch advances ndom independent D2Q9 lattices (the benchmark geometries
 * of Sec. V, e.g. sweeps over kappa_m and h_m) together.  Each domain has its
 * own tlb_params (lattice TLB_D2Q9, nx, ny <= 65535, its own walls_y, kappa,
 * alpha, tau and Gamma); every domain must use the same prec.  One time step
 * of the batch is one persistent kernel launch per stream group (one group
 * unless tlb_batch_set_launch asks for more) whose workgroups take
 * (domain, strip, row-chunk) or (domain, run of positions) work items from
 * per-XCD queues; with tlb_batch_set_graph the steps are replayed from
 * captured hipGraphs (one per group).
 * A domain evolves exactly (bit for bit) as a tlb_sim with the same
 * parameters.  Domain indices run 0..ndom-1; host arrays follow the layouts
 * of the single-lattice calls for that domain's nx, ny.
 */
typedef struct tlb_batch tlb_batch;
tlb_status tlb_batch_create(const tlb_params* per_dom, int32_t ndom, void* stream, tlb_batch** out);
tlb_status tlb_batch_destroy(tlb_batch* batch);
int32_t tlb_batch_size(const tlb_batch* batch);
/* Total number of fluid nodes over all domains. */
int64_t tlb_batch_nodes(const tlb_batch* batch);
void* tlb_batch_get_stream(const tlb_batch* batch);
tlb_status tlb_batch_synchronize(tlb_batch* batch);
/* Wetting parameters of one wall of one domain (host [3][nx]); values outside
 * |4 h_m / (alpha kappa_m)| <= 1 are applied as given and counted as for
 * tlb_set_wetting (one stderr warning per batch);
 * tlb_batch_wetting_outside_range gives the count of one domain, or of all
 * domains for dom = -1. */
tlb_status tlb_batch_set_wetting(tlb_batch* batch, int32_t dom, int wall, const double* h);
tlb_status tlb_batch_wetting_outside_range(const tlb_batch* batch, int32_t dom, int64_t* count);
tlb_status tlb_batch_init_equilibrium(tlb_batch* batch, int32_t dom, const double* C, const double* u);
tlb_status tlb_batch_step(tlb_batch* batch, int64_t nsteps);
tlb_status tlb_batch_get_field(tlb_batch* batch, int32_t dom, int which, double* out);
tlb_status tlb_batch_get_populations(tlb_batch* batch, int32_t dom, int species, double* out);
tlb_status tlb_batch_diagnostics(tlb_batch* batch, int32_t dom, tlb_diag* out);
/*
 * Launch shape of the batched step: width = workgroup width (64, 128, 256);
 * variant 0 and 1 sweep every domain in strips of that many columns, chunk =
 * rows per work item (1 adds a one-row prefetch, as for a D2Q9 tlb_sim);
 * variant 2 sweeps each domain with nx + 3 <= width as one flat sequence of
 * its rows (each padded with its two periodic halo columns), chunk = runs of
 * `width` consecutive positions per work item, so that narrow domains leave
 * no lanes idle, and the wider domains in strips as variant 0.  chunk is
 * 1..65535.  height (1..4, 0 means 1) splits the domains into that many
 * stream groups of nearly equal work (at most one per domain); each group
 * runs its own chain of launches on its own stream, forked from and joined
 * back into the batch's stream inside tlb_batch_step, so that one group's
 * launch fills the compute units another group's launch leaves idle as it
 * drains.  With more than one group every group runs on a stream the
 * library creates (four, together, at the default priority).  Results do
 * not depend on the shape.
 */
tlb_status tlb_batch_set_launch(tlb_batch* batch, const tlb_launch* launch);
tlb_status tlb_batch_get_launch(const tlb_batch* batch, tlb_launch* out);
/*
 * Time every launch shape for trial_steps steps from the current state
 * (which is restored) in one stream group, then the fastest of them in 1, 2,
 * 3 and 4 groups, each with its chunk and with twice and four times its
 * chunk, for 4 * trial_steps steps each, and keep the fastest of those;
 * writes it to *chosen if not NULL.
 * If the environment variable TLB_TUNE_CACHE names a file, a previous result
 * for the same domain sizes is taken from it, and new results are appended.
 */
tlb_status tlb_batch_autotune(tlb_batch* batch, int32_t trial_steps, tlb_launch* chosen);
/* Capture steps_per_graph (even, > 0) steps once in a hipGraph and replay it
 * inside tlb_batch_step; 0 launches every step directly (the default). */
tlb_status tlb_batch_set_graph(tlb_batch* batch, int32_t steps_per_graph);

#ifdef __cplusplus
}
#endif

#endif /* TLB_H */
