/*
 * tild.h -- C ABI of libtild, a gfx950 (MI355X) implementation of one
 * theoretically-informed Langevin dynamics (TILD) step: the particle-mesh
 * non-bonded force of a two-species (A/B) bead-spring melt (optionally with
 * smeared electrostatics), harmonic bond forces, and an overdamped
 * Euler-Maruyama (or GJF Langevin) position update; with energy gradients,
 * Hessian-vector products and mesh access for differentiable use, and
 * batches of independent systems stepped together.
 *
 * Model (MATILDA.FT paper, Sec. "Structure of theoretically-informed
 * coarse-grained and field-theoretic models"):
 *   - microscopic densities rho_K = sum_j delta(r - r_j), Eq. rhohat;
 *   - bonds beta U_0 = sum 3/(2 b^2) |r_s - r_{s+1}|^2, Eq. bonds
 *     (here U = bond_k |d|^2, d the minimum-image bond vector);
 *   - Flory term (chi/rho_0) int int rho_A u_G rho_B, Eq. fh, and Helfand
 *     term (kappa/2 rho_0) int int (rho_+ - rho_0) u_G (rho_+ - rho_0),
 *     Eq. HelfandP, with rho_0 = N/V and u_G a unit Gaussian of variance
 *     sigma^2 = 2 a^2, i.e. u_G = h * h for the smearing h of width a
 *     (Eqs. smearRho, fhF, HelfandF); its transform is exp(-a^2 k^2).
 * Electrostatics (Sec. "Long-range interactions": the same mesh carries the
 * forces between charged monomers; Sec. "Input Script": one Bjerrum length
 * and one charge spreading length): with per-species charges q_K the pair
 * kernel of species K and L gains q_K q_L (4 pi l_B / V) exp(-a_e^2 k^2) / k^2
 * (k = 0 left out: a neutralising background), i.e. the energy
 * E_e = (l_B / 2) int int rho_e~ rho_e~ / |r - r'| of the smeared charge
 * density, so it rides through the same spread, transforms and gather.
 * Method (Sec. "Long-range interactions", Eq. PMM, Fig. pmm): beads are
 * assigned to a periodic grid with order-P B-spline weights, the species
 * densities are Fourier transformed, multiplied by the kernel and by i k,
 * transformed back to field gradients and interpolated to the beads with the
 * same weights.  Integrators (Sec. "Integrator Class"): Euler-Maruyama with
 * internally generated noise, in the overdamped form of Eq. EM (default), or
 * the Gronbech-Jensen--Farago (GJF) Langevin scheme (TILD_INTEGRATOR_GJF).
 *
 * Conventions shared by every call:
 *   - Units: kT, bead mass and the segment length b are the reduced units of
 *     the paper (Sec. "Units").
 *   - Box: orthogonal, fully periodic, edges box[0..2] > 0.  Positions are
 *     wrapped into [0, L).  Internally they are stored as 32-bit unsigned
 *     fixed-point fractions of the box (resolution L / 2^32).
 *   - Grid nodes sit at g * L/M from the box corner.  order = P is the number
 *     of grid points per dimension touched by a bead (P = 2 is the paper's
 *     "two nearest grid points" first-order scheme); weights are the
 *     centred cardinal B-spline of order P.
 *   - Non-bonded force: ik route (default); the derivative wavenumber is zero
 *     on the Nyquist plane of an even grid axis, so the net non-bonded force
 *     is zero.  TILD_FORCE_AD selects the exact gradient of the mesh energy.
 *   - Noise: Philox4x32-10 (Salmon et al., SC'11) with key (seed mod 2^32,
 *     seed >> 32) and counter (bead id, step mod 2^32, step >> 32, 0); the
 *     four words map to uniforms (w + 1/2) 2^-32 and Box-Muller gives the
 *     x, y (from words 0, 1) and z (from words 2, 3) increments.  Bead id is
 *     the bead's index in the arrays given to tild_create, so a run resumed
 *     from (positions, step count, seed) continues the same noise stream.
 *   - Bead order in every input and output array is the order of the types
 *     array given to tild_create ("ABI order").
 *
 * Ownership: the caller owns every pointer it passes.  Input arrays are
 * copied (or fully consumed) before the call returns and may be freed
 * immediately after.  Output arrays are allocated by the caller.  The
 * context owns all device memory it allocates and frees it in tild_destroy.
 *
 * Streams: all device work of a context is enqueued on the HIP stream given
 * to tild_create (NULL = the null stream).  tild_step is asynchronous; calls
 * that return host data (tild_energy, and tild_get_positions / tild_forces
 * with on_device = 0) synchronise that stream.  Device-pointer inputs and
 * outputs must be valid on the context's device and are read/written in
 * stream order.
 *
 * Errors: every int-returning call returns TILD_OK (0) or a negative code.
 * The message of the last failure is available from tild_last_error.  No C++
 * exception crosses this interface.  A non-finite force or displacement seen
 * during tild_step is latched on the device and reported as TILD_ENONFINITE
 * by the next synchronising call (tild_synchronize, tild_energy, or a
 * host-output call); the flag is then cleared.  So is a grid plane too dense
 * for the fixed-point spread (of the order of 10^7 beads reaching one
 * plane of one species).  An internal consistency failure latched on the
 * device (a bead outside its bin, a prefix scan that gave up waiting) is
 * reported the same way as TILD_EHIP.
 */
#ifndef TILD_H
#define TILD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define TILD_OK 0
#define TILD_EINVAL (-1)     /* bad argument: NULL pointer, parameter out of range, bond index out of range */
#define TILD_ENOMEM (-2)     /* a device or host allocation failed */
#define TILD_EHIP (-3)       /* a HIP runtime call failed; the HIP error string is in tild_last_error */
#define TILD_ENONFINITE (-4) /* NaN/Inf force or displacement detected during a step */
#define TILD_ESTATE (-5)     /* call not valid in the current state (e.g. no positions set) */

/* Arithmetic precision of grids, transforms and forces (tild_params.precision)
 * and element type of position / force arrays (dtype arguments). */
#define TILD_FP32 0
#define TILD_FP64 1

/* tild_params.flags */
#define TILD_COM_CORRECT 1u /* subtract the mean displacement of every step (centre-of-mass drift correction) */
#define TILD_POTENTIAL_SAMPLED 2u /* kernel u^ = dV x DFT of the smearing Gaussian u_G sampled at the
                                     minimum-image node separations (the potential built by FFT and stored,
                                     Sec. "Long-range interactions"), instead of the analytic exp(-a^2 k^2);
                                     needs smear_a > 0.  Energies use it (including the k = 0 constant
                                     chi N_A N_B u^(0) / N); the virial keeps the analytic kernel. */
#define TILD_FORCE_AD 8u /* non-bonded force by the exact gradient of the mesh energy,
                           F_i = -sum_g grad_i W_i(g) phi_{s_i}(g) with the potential fields phi_K
                           (2 inverse transforms instead of 6), instead of the ik route of Eq. PMM;
                           needs order >= 2.  Its net force is not exactly zero: with
                           TILD_COM_CORRECT the mean force enters the mean displacement. */
#define TILD_INTEGRATOR_GJF 16u /* GJF Langevin integrator (Gronbech-Jensen and Farago, Mol. Phys. 111, 983
                                   (2013)) with bead mass `mass`, friction gamma and noise
                                   beta_n = sqrt(2 gamma kT dt) xi(step n).  Each step applies
                                     D_{n+1} = a D_n + (b dt^2 / m) F_n + (b dt / 2m) (beta_n + beta_{n+1}),
                                     x_{n+1} = x_n + D_{n+1},
                                   c = gamma dt / 2m, a = (1 - c)/(1 + c), b = 1/(1 + c): the velocity
                                   form of the scheme with the on-site velocity eliminated.  The state
                                   carried between steps is the half-step velocity
                                   u = D / (sqrt(b) dt) (tild_set_velocities, tild_get_velocities; zero
                                   at creation).  With TILD_COM_CORRECT the mean of D is removed. */
#define TILD_DETERMINISTIC 4u /* accepted for compatibility: steps, forces and energies are already bitwise
                                 reproducible run to run (the spread accumulates fixed-point integers in
                                 both precisions, every reduction has a fixed order).  The directional and
                                 weighted counts of tild_hvp, tild_force_vjp and tild_adjoint_step are
                                 summed with floating-point atomics: those results vary at the rounding
                                 level (about 1e-13 relative in FP64) */

/* tild_forces parts */
#define TILD_PART_NONBONDED 1u
#define TILD_PART_BOND 2u
#define TILD_PART_TOTAL 3u

/* Per-kernel timing slots reported by tild_profile_steps. */
#define TILD_NUM_KERNELS 6

typedef struct tild_ctx tild_ctx;

typedef struct tild_params {
    double box[3];     /* L_x, L_y, L_z > 0 (orthogonal periodic box) */
    int32_t grid[3];   /* M_x, M_y, M_z: each 2..256 and a product of 2, 3 and 5 only */
    int32_t order;     /* P, grid points per dimension of the assignment stencil: 1..7, P <= min(M) */
    double smear_a;    /* smearing width a >= 0: kernel transform exp(-a^2 k^2) */
    double chi;        /* Flory-Huggins chi_AB (Eq. fh) */
    double kappa;      /* Helfand compressibility kappa (Eq. HelfandP) */
    double bond_k;     /* bond energy bond_k |d|^2 per bond; 3/(2 b^2) = 1.5 at b = 1 (Eq. bonds) */
    double dt;         /* time step > 0 */
    double gamma;      /* friction > 0; mobility 1/gamma */
    double kT;         /* temperature >= 0 (noise amplitude sqrt(2 kT dt / gamma)) */
    uint64_t seed;     /* Philox key */
    int32_t precision; /* TILD_FP32 (float grids, transforms and forces; float64 energy, virial and
                          centre-of-mass sums) or TILD_FP64 (everything in float64) */
    uint32_t flags;    /* TILD_COM_CORRECT, TILD_POTENTIAL_SAMPLED, TILD_FORCE_AD, TILD_INTEGRATOR_GJF,
                          TILD_DETERMINISTIC, or 0 */
    double mass;       /* bead mass for TILD_INTEGRATOR_GJF (> 0; 0 is read as 1); unused by Euler-Maruyama */
    double charge[2];  /* charge of an A and of a B bead (elementary charges); electrostatics is on when
                          bjerrum != 0 and a charge is non-zero */
    double bjerrum;    /* Bjerrum length l_B >= 0 (Coulomb energy l_B / r kT between unit point charges) */
    double charge_smear; /* charge spreading length a_e >= 0: charges are Gaussian clouds of width a_e, as
                            the mass density is smeared with width a (Eq. smearRho) */
} tild_params;

/*
 * Device bytes a context for these parameters and bonds needs: the size of a
 * caller workspace for tild_create.  bonds as for tild_create (the partner
 * table is as wide as the largest bead degree).  Touches no device.  Returns
 * 0 when the arguments are invalid (the reason is in tild_last_error(NULL)).
 */
size_t tild_workspace_bytes(const tild_params* params, int64_t n_beads, int64_t n_bonds, const int32_t* bonds);

/*
 * Create a context for n_beads beads.
 *   types:  host array [n_beads] of int32, 0 = species A, 1 = species B.
 *   bonds:  host array [2 * n_bonds] of int32 pairs (i, j), 0-based ABI
 *           indices, i != j; may be NULL when n_bonds == 0.
 *   workspace, workspace_bytes: NULL, or device memory on the current device,
 *           256-byte aligned, of at least tild_workspace_bytes(...) bytes,
 *           owned by the caller and kept alive until tild_destroy; the
 *           context then takes all its device buffers from it and allocates
 *           no device memory (TILD_ENOMEM when it is too small).  NULL: the
 *           library allocates and frees its own.
 *   hip_stream: a hipStream_t on the current device, or NULL.
 * Positions must be set with tild_set_positions before the first step,
 * force or energy call.  The step counter starts at 0.
 * Returns TILD_EINVAL for invalid parameters (grid not 2,3,5-smooth or out
 * of range, order out of range, non-positive box/dt/gamma, NULL arrays, bond
 * index out of range, types other than 0/1, a grid plane too large for one
 * workgroup's local memory in the chosen precision, a workspace not 256-byte
 * aligned), TILD_ENOMEM or TILD_EHIP.  On failure *out is set to NULL and
 * the message is available from tild_last_error(NULL) on the same thread.
 */
int tild_create(const tild_params* params, int64_t n_beads, const int32_t* types,
                int64_t n_bonds, const int32_t* bonds, void* workspace, size_t workspace_bytes,
                void* hip_stream, tild_ctx** out);

/*
 * Set all positions.  xyz: [n_beads][3] in ABI order, element type dtype
 * (TILD_FP32 or TILD_FP64), host memory (on_device = 0) or device memory
 * (on_device = 1).  Coordinates may lie outside the box; they are wrapped.
 * Non-finite coordinates give TILD_EINVAL (host input) or TILD_ENONFINITE at
 * the next synchronising call (device input).  Does not change the step
 * counter.
 */
int tild_set_positions(tild_ctx* ctx, const void* xyz, int32_t dtype, int32_t on_device);

/* Copy the current positions, wrapped into [0, L), to xyz ([n_beads][3], ABI order). */
int tild_get_positions(tild_ctx* ctx, void* xyz, int32_t dtype, int32_t on_device);

/*
 * Half-step velocities of a TILD_INTEGRATOR_GJF context: u = (x_n - x_{n-1}) /
 * (sqrt(b) dt) of the last step (Gronbech-Jensen, Jensen and Farago, Mol.
 * Phys. 118, e1662506 (2020): for a free particle its variance is exactly
 * kT/m at any dt), which the next step uses as D_n = sqrt(b) dt u.
 * v: [n_beads][3] in ABI order, dtype element type, host or device memory.
 * Positions must have been set (TILD_ESTATE otherwise); a context without
 * TILD_INTEGRATOR_GJF gives TILD_EINVAL.  tild_set_positions keeps every
 * bead's velocity.  Non-finite host input gives TILD_EINVAL.
 */
int tild_set_velocities(tild_ctx* ctx, const void* v, int32_t dtype, int32_t on_device);
int tild_get_velocities(tild_ctx* ctx, void* v, int32_t dtype, int32_t on_device);

/*
 * Enqueue n_steps >= 0 steps.  Each step evaluates the forces at the current
 * positions (non-bonded + bonds) and applies
 *   x <- wrap(x + (dt/gamma) F + sqrt(2 kT dt/gamma) xi - Delta),
 * Delta being the mean displacement when TILD_COM_CORRECT is set, xi the
 * Philox noise of the current step index (with TILD_INTEGRATOR_GJF the GJF
 * update given with that flag instead); the step counter then advances.
 * Asynchronous: returns after enqueueing.
 */
int tild_step(tild_ctx* ctx, int64_t n_steps);

/*
 * Forces at the current positions, without moving the beads.
 *   out: [n_beads][3] in ABI order, dtype element type, host or device memory.
 *   parts: TILD_PART_NONBONDED, TILD_PART_BOND or TILD_PART_TOTAL (their sum).
 */
int tild_forces(tild_ctx* ctx, void* out, int32_t dtype, int32_t on_device, uint32_t parts);

/*
 * Non-bonded forces (the context's route) at the current positions with chi
 * and kappa replaced by the given values; the smearing, the kernel and the
 * context's own parameters are unchanged, and with_charges = 0 leaves the
 * electrostatic part out.  The forces are linear in chi and kappa, so
 * (1, 0, 0) and (0, 1, 0) give dF/dchi and dF/dkappa (adjoints through time
 * steps).  out as for tild_forces.
 */
int tild_interaction_forces(tild_ctx* ctx, double chi, double kappa, int32_t with_charges, void* out,
                            int32_t dtype, int32_t on_device);

/*
 * Energies (kT) and virial at the current positions, accumulated in float64:
 *   out[0] E_bond, out[1] E_chi, out[2] E_kappa, out[3] E_total,
 *   out[4..6] W_xx, W_yy, W_zz with W_aa = -L_a dE/dL_a at fixed scaled
 *   coordinates (bonded + non-bonded), out[7] E_elec (0 without charges;
 *   included in E_total).
 * E_chi includes the constant k = 0 term chi N_A N_B / N; both non-bonded
 * terms include the grid-dependent bead self-interaction.  Synchronises.
 */
int tild_energy(tild_ctx* ctx, double out[8]);

/*
 * Energy and its gradients at the current positions (the differentiable
 * form of Eqs. fh, HelfandP and bonds).  Synchronises.
 *   out[0] E_total; out[1] dE/dchi = (1/N) sum_n u^ Re(c^_A* c^_B);
 *   out[2] dE/dkappa = (1/2N) sum_{n!=0} u^ |c^_A + c^_B|^2;
 *   out[3] dE/da = sum_n -2 a k^2 u^ [...] (analytic kernel; NaN with
 *   TILD_POTENTIAL_SAMPLED), all at fixed positions.
 *   grad_x: NULL, or [n_beads][3] (ABI order, dtype, host or device) that
 *   receives dE/dx = -(F_nb + F_bond) with F_nb the exact gradient of the
 *   mesh energy (whatever route tild_step uses); needs order >= 2.
 */
int tild_energy_grad(tild_ctx* ctx, double out[4], void* grad_x, int32_t dtype, int32_t on_device);

/*
 * Change chi, kappa and the smearing width a of an existing context (for
 * differentiating through them); smear_a >= 0, > 0 with
 * TILD_POTENTIAL_SAMPLED.  Waits for the context's queued work first.
 */
int tild_set_interaction(tild_ctx* ctx, double chi, double kappa, double smear_a);

/* Number of steps taken since creation (or since tild_set_step_count). */
int64_t tild_step_count(const tild_ctx* ctx);

/* Set the step counter (the noise stream position), e.g. to resume a run. */
int tild_set_step_count(tild_ctx* ctx, int64_t step);

/* Wait for the context's stream; report a latched non-finite flag. */
int tild_synchronize(tild_ctx* ctx);

/* Free the context and all device memory it owns.  NULL is a no-op. */
void tild_destroy(tild_ctx* ctx);

/* Message of the last failure on ctx, or of the last failed tild_create on
 * this thread when ctx is NULL.  Valid until the next call on ctx. */
const char* tild_last_error(const tild_ctx* ctx);

/*
 * Instrumented steps for measurement: runs n_steps steps exactly like
 * tild_step, with a HIP event pair recorded on the context's stream around
 * every kernel launch, then synchronises and writes the mean duration in
 * milliseconds of each kernel slot to kernel_ms[0 .. n_slots-1] (n_slots <=
 * TILD_NUM_KERNELS) and the launches per step of each slot to
 * launches_per_step (may be NULL; the update slot holds two launches on the
 * exact-gradient route, the shift reduction and the update).  Slot names: tild_kernel_name(slot).
 */
int tild_profile_steps(tild_ctx* ctx, int64_t n_steps, double* kernel_ms,
                       int32_t* launches_per_step, int32_t n_slots);

/* Name of a kernel timing slot, or NULL when slot is out of range. */
const char* tild_kernel_name(int32_t slot);

/*
 * Device-to-device copy of `bytes` bytes (a multiple of 16) with the
 * library's own streaming kernel, repeated `iters` times on `hip_stream`;
 * writes the mean milliseconds per copy.  Used to calibrate achievable HBM
 * bandwidth and hardware byte counters.  dst and src must not overlap.
 */
int tild_stream_copy(void* dst, const void* src, size_t bytes, int32_t iters,
                     void* hip_stream, double* ms_per_copy);

/*
 * Grid access for losses and external fields (differentiable use).  Grid
 * arrays are [2][M_z][M_y][M_x] (species, then z, y, x with x fastest) in the
 * context's working precision (float for TILD_FP32, double for TILD_FP64),
 * host or device memory (on_device).
 * tild_counts: the assignment counts c_K(g) = sum_{i in K} W_i(g) at the
 *   current positions (density c_K / dV, Eq. rhohat on the mesh).
 * tild_field_forces: the forces -sum_g grad W_i(g) psi_{s_i}(g) of a given
 *   field psi (the gradient of sum_g c_K(g) psi_K(g), i.e. of any loss whose
 *   derivative by the counts is psi), out [n_beads][3] ABI order, dtype;
 *   field and out both host or both device memory.  Needs order >= 2.
 * Host calls synchronise.
 */
int tild_counts(tild_ctx* ctx, void* out, int32_t on_device);
int tild_field_forces(tild_ctx* ctx, const void* field, void* out, int32_t dtype, int32_t on_device);

/*
 * Hessian-vector product of the total energy (mesh energy of Eqs. fh,
 * HelfandP and electrostatics, plus bonds) at the current positions:
 *   out_i = sum_j (d^2 E / dx_i dx_j) v_j
 *         = sum_g (grad grad W_i(g)) v_i phi_{s_i}(g) + sum_g grad W_i(g) delta phi_{s_i}(g) + (H_b v)_i,
 * delta phi the potential of the directional counts sum_j grad W_j . v_j,
 * H_b v the bond term 2 bond_k sum_partners (v_i - v_j).  -H v is the
 * Jacobian of the exact-gradient force applied to v, and also its transpose
 * (H is symmetric), the building block of adjoints through time steps.
 * v, out: [n_beads][3] in ABI order, dtype, both host or both device
 * memory (on_device).  Needs order >= 3 (TILD_EINVAL otherwise).  Host
 * calls synchronise.
 */
int tild_hvp(tild_ctx* ctx, const void* v, void* out, int32_t dtype, int32_t on_device);

/*
 * Transposed Jacobian of the context's force at the current positions:
 *   out = (dF/dx)^T lam,  F = the non-bonded force of the context's route plus the bond force.
 * On the ik route (Eq. PMM with Eq. bonds; F^ik is not the gradient of an
 * energy, so dF/dx is not symmetric) this is
 *   out_j = -sum_a lam_j,a sum_g grad W_j(g) d_a phi_{s_j}(g)          (the weights move with bead j)
 *           + sum_g grad W_j(g) psi_{s_j}(g)                            (the field moves with every bead)
 *           - (H_b lam)_j,
 * psi = sum_a d_a phi^(a), phi^(a) the field of the counts sum_i lam_i,a W_i
 * (the derivative operators i k^D are antisymmetric, the pair kernel
 * symmetric); on the exact-gradient route it is -H lam (tild_hvp).
 * lam, out: [n_beads][3] in ABI order, dtype, both host or both device
 * memory (on_device).  Needs order >= 2 (ik) or >= 3 (exact gradient),
 * TILD_EINVAL otherwise.  Host calls synchronise.
 */
int tild_force_vjp(tild_ctx* ctx, const void* lam, void* out, int32_t dtype, int32_t on_device);

/*
 * One backward step of the adjoint of Euler-Maruyama steps (Eq. EM with the
 * context's force and its noise held fixed), at the current positions x_t:
 *   dtheta[0] += (dt/gamma) (Pr lam) . dF/dchi(x_t),
 *   dtheta[1] += (dt/gamma) (Pr lam) . dF/dkappa(x_t),
 *   lam       <- lam + (dt/gamma) (dF/dx)(x_t)^T Pr lam,
 * Pr removing the mean over the beads when TILD_COM_CORRECT is set; dF/dchi
 * and dF/dkappa are the non-bonded forces with (chi, kappa) = (1, 0) and
 * (0, 1) and no charges (the force is linear in both).  Run backwards over
 * t = K-1 .. 0 from lam = dL/dx_K it gives dL/dx_0 and dL/d(chi, kappa).
 *   lam:    device [n_beads][3] float64, ABI order, updated in place.
 *   dtheta: device float64[2], added to.
 * Asynchronous on the context's stream; its own sums run in a fixed order,
 * while the transposed Jacobian accumulates grid counts with floating-point
 * atomics (results vary at the rounding level).  Euler-Maruyama contexts
 * with order >= 2 (ik) or >= 3 (exact gradient).
 */
int tild_adjoint_step(tild_ctx* ctx, double* lam, double* dtheta);

/*
 * Batches: independent contexts (replicas of uneven box, grid and bead
 * count: the multiple boxes of replica exchange, parallel tempering or Gibbs
 * ensemble sampling the paper plans, Sec. "Planned future developments")
 * stepped together, one launch per
 * kernel for all members instead of one per member.
 *   ctxs: n_ctx >= 1 distinct contexts on the current device, all with the
 *         same precision, order and flags, all charged or all neutral, on
 *         the ik route with Euler-Maruyama (no TILD_FORCE_AD, no
 *         TILD_INTEGRATOR_GJF); at most 16,776,960 beads each.  The batch
 *         borrows them: they must outlive it.
 *   hip_stream: the stream the batch's work is enqueued on (NULL = null stream).
 * tild_batch_step advances every member by n_steps (< 2^31) steps, exactly as
 * tild_step on each member would (same noise stream, same step counters), and
 * returns after enqueueing.  The batch's stream first waits for the work
 * queued on each member's stream, and each member's stream then waits for
 * the batch, so calls on a member (positions, forces, energy) stay ordered
 * with the batch.  It also waits on the host until the previous call's
 * descriptor upload (a few hundred bytes per member) has been read.
 * TILD_ESTATE if a member's positions were never set.
 * tild_batch_synchronize waits for the batch's stream and reports the first
 * member's latched error (as tild_synchronize).  Errors of a batch call are
 * described by tild_batch_last_error (creation errors: tild_batch_last_error(NULL)).
 */
typedef struct tild_batch tild_batch;
int tild_batch_create(tild_ctx* const* ctxs, int32_t n_ctx, void* hip_stream, tild_batch** out);
int tild_batch_step(tild_batch* batch, int64_t n_steps);
/*
 * Choose the batch's plane-workgroup size (256 or 512 threads; the default
 * is set from the largest member plane) by timing trial_steps (1..1000)
 * batched steps with each, twice, on the members' own systems with eager
 * launches; then, with that size, the column block of the k-space pass
 * (each member's own, or 8, 12, 16, 24 or 32 columns for every member,
 * widths whose local memory does not fit skipped; twice each); then whether
 * replaying the steps from a captured HIP graph is faster.  Every member's
 * positions and step counter are restored after each trial, so the
 * simulation state is unchanged (bitwise: the column block changes no
 * result).  Synchronises; needs a temporary device buffer of 24 bytes per
 * bead and rebuilds the batch's work-unit maps.  The choices are stored in
 * *plane_block (threads), *z_cols (0 = each member's own) and *graph (1 =
 * graph replay) when those are not NULL.
 */
int tild_batch_autotune(tild_batch* batch, int32_t trial_steps, int32_t* plane_block, int32_t* z_cols,
                        int32_t* graph);
/*
 * Replay batched steps from captured HIP graphs (use_graph != 0, the default)
 * or launch every kernel of every step from the host (0).  With graphs, the
 * first call asking for n_steps steps captures them (every batched kernel of
 * every step, on a private stream) and later calls of that many steps
 * replay the graph after uploading the members' descriptors; a change of
 * step count or plane-workgroup size captures again.
 */
int tild_batch_set_graph(tild_batch* batch, int32_t use_graph);
int tild_batch_synchronize(tild_batch* batch);
void tild_batch_destroy(tild_batch* batch);
const char* tild_batch_last_error(const tild_batch* batch);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): step
 * n_ctx contexts as one batch, exactly as tild_batch_create + tild_batch_step
 * + tild_batch_destroy would (bitwise the same positions), without a batch
 * object and without allocating anything.  The member descriptors, the
 * work-unit maps and the bin-scan status words go into a fixed 1 MiB
 * scratch array that the library holds on each device until the process
 * ends (its address is taken on the first call on that device); a batch
 * that needs more (a few hundred bytes per member plus 4 bytes per work
 * unit: about 280 KB for 64 replicas of 5.8 million beads in all) is
 * rejected with TILD_EINVAL.
 *   ctxs: as for tild_batch_create; every member must have been created on
 *         hip_stream (TILD_EINVAL otherwise), and the work is enqueued there.
 *   n_steps: 0 .. 2^31 - 1.  TILD_ESTATE if a member's positions were never set.
 * Returns after enqueueing (the host waits only for the previous call's
 * upload of the maps to have been read).  Calls on one device share the
 * scratch array and keep the last call's contents: calls whose work
 * overlaps on the device (different streams, no ordering) race.  Errors are
 * described by tild_batch_last_error(NULL).
 */
int tild_batch_step_static(tild_ctx* const* ctxs, int32_t n_ctx, int64_t n_steps, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* TILD_H */
