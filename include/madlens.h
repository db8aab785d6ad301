/*
 * madlens.h -- C ABI of libmadlens_amd.so, the MI355X (gfx950) hot path of
 * the MADLens differentiable lensing simulator (Boehm, Feng, Lee, Dai,
 * arXiv 2012.07266).
 *
 * The library runs a FastPM particle-mesh simulation from Gaussian initial
 * modes and projects the particles of every step, weighted by the lensing
 * kernel, onto convergence maps at a list of source redshifts (package
 * design section and the parameter table of the paper).  It also provides
 * vector-Jacobian products with respect to the initial white-noise modes,
 * Omega_m and sigma_8 (package design section; appendix on cosmology
 * derivatives).
 *
 * Conventions shared by every entry point
 *  - Every call returns an int: PM_OK (0) or a negative PM_E* code.  Nothing
 *    throws across the ABI.  pm_strerror() names a code.
 *  - Pointers named "device" are HIP device addresses.  The caller owns every
 *    buffer it passes; the library never keeps a caller pointer past the
 *    call, except the stream handle given to pm_create.
 *  - All device work is enqueued on the stream given to pm_create and is
 *    asynchronous with respect to the host; pm_sync() waits for it.
 *  - The library allocates all device memory it uses in pm_create (the
 *    "arena"); no later call allocates or frees device memory.
 *  - Caller buffers hold elements of the simulation's dtype: float for
 *    PM_F32, double for PM_F64.
 *  - A pm_sim is used by one host thread at a time.
 *  - Units: lengths in Mpc/h, wave numbers in h/Mpc, map sizes in degrees.
 *    Positions are in [0, box); momenta are p = a^3 E(a) dx/da in Mpc/h,
 *    with E = H/H0.
 *  - Particle arrays are [3][Np^3] in lattice order: particle
 *    (i0, i1, i2) is element (i0 * Np + i1) * Np + i2, C order.
 *  - Meshes are [Nm][Nm][Nm] in C order, last axis contiguous.
 *  - Maps are [nsrc][npix][npix]; map[s][j0][j1] covers theta_0 (first axis,
 *    along box axis 0) and theta_1 (along box axis 1), centred on the line of
 *    sight, which runs along box axis 2 from an observer at (L/2, L/2, 0).
 */
#ifndef MADLENS_H
#define MADLENS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define PM_OK           0
#define PM_EINVAL      -1   /* invalid argument or unsupported size          */
#define PM_ENOMEM      -2   /* device arena could not be allocated           */
#define PM_EDEVICE     -3   /* a HIP runtime call failed                     */
#define PM_ESTATE      -4   /* the simulation is not in the required state   */
#define PM_ENONFINITE  -5   /* a kernel produced a non-finite position       */
#define PM_EAGAIN      -7   /* not finished yet (serving)                    */
#define PM_ETOOBIG     -8   /* beyond pm_run_noalloc's static scratch        */
#define PM_EFULL       -9   /* every slot of a batch is taken                */

#define PM_F32 0
#define PM_F64 1

/* ---- parameters (the paper's parameter table) -------------------------- */
typedef struct pm_params {
    int32_t np;        /* particles per side, Np                             */
    int32_t nm;        /* force-mesh cells per side, Nm = B * Np, B in {1,2}  */
    double  box;       /* periodic box side L, Mpc/h                          */
    double  omega_m;   /* total matter density today, flat: OL = 1 - Om      */
    double  omega_b;   /* baryon density (Eisenstein-Hu transfer shape)      */
    double  h;         /* H0 / (100 km/s/Mpc)                                */
    double  n_s;       /* primordial spectral index                          */
    double  sigma8;    /* rms linear fluctuation in 8 Mpc/h spheres at a = 1 */
    double  t_cmb;     /* CMB temperature, K                                 */
    int32_t dtype;     /* PM_F32 or PM_F64: precision of every kernel        */
    uint32_t modes;    /* PM_MODE_* bits: optional passes whose buffers the
                          arena must hold (0: forward and reverse only)     */
} pm_params;

/* Optional passes of a handle.  Their device buffers are part of the arena
 * that pm_create allocates and pm_footprint counts; a call that needs a
 * mode the handle was created without fails with PM_EINVAL. */
#define PM_MODE_PGD     1u  /* pm_set_pgd: filter table, shift [3][Np^3] and
                               one spare mesh [Nm^3] + Nyquist plane         */
#define PM_MODE_TANGENT 2u  /* forward-mode tangents: 15 Np^3 values         */
#define PM_MODE_CKPT_FORCE 4u /* checkpoints also carry the force at the saved
                               state (three force meshes [3][Nm^3] and the
                               particles' accelerations [3][Np^3]), so that
                               pm_checkpoint_load restores it, bit for bit,
                               instead of recomputing it (a paint, the force
                               transform and a readout); no arena buffers   */

typedef struct lens_params {
    int32_t       npix;     /* map pixels per side                           */
    double        fov_deg;  /* map side in degrees, (0, 22]                  */
    int32_t       nsrc;     /* number of source planes (maps), 1..16         */
    const double* z_src;    /* host array [nsrc] of source redshifts, copied */
} lens_params;

typedef struct pm_sim pm_sim;

/* Size rules: Nm and Np are multiples of 16 (Np >= 16), Nm / Np is 1 or 2,
 * Nm and Np have no prime factor other than 2 and 3 and are at most 1024;
 * 0 < Omega_m < 1; box > 0; 16 <= npix <= 8192; modes holds no bit other
 * than the PM_MODE_* ones.  Violations give PM_EINVAL. */

/* Bytes of device memory pm_create would allocate for these parameters; 0
 * when they are invalid.  Pure host function (used for admission by HBM
 * footprint in serving). */
size_t pm_footprint(const pm_params* p, const lens_params* l);

/* Validate parameters, build the float64 background tables (comoving
 * distance, growth, lensing-weight tables, the Eisenstein-Hu no-wiggle
 * linear spectrum normalised to sigma8) and allocate the whole device arena.
 * `hip_stream` is a hipStream_t (NULL = the default stream).
 * On success *out owns the arena until pm_destroy.
 * Errors: PM_EINVAL, PM_ENOMEM, PM_EDEVICE. */
int pm_create(const pm_params* p, const lens_params* l, void* hip_stream,
              pm_sim** out);

/* Free the arena and the handle.  PM_EINVAL on NULL. */
int pm_destroy(pm_sim* sim);

/* Zel'dovich (first-order LPT) initial conditions at scale factor a0 from
 * Gaussian white noise (package design section: derivatives are taken with
 * respect to these initial Gaussian modes; appendix: LPT initial
 * conditions).  `noise` is a device array [Np^3] of N(0,1) values in
 * lattice order.  delta_hat = rfft(noise) sqrt(P(k) Np^3 / L^3), displacement
 * s_hat_j = i k_j delta_hat / k^2, x0 = q + D(a0) s, p0 = g_p(a0) s, with the
 * lattice point q = (B i + 1/2) L / Nm.  Also computes the force at x0.
 * Errors: PM_EINVAL (NULL noise, a0 not in (0, 1], or chi(a0) closer than the
 * farthest source plane). */
int pm_init_ic(pm_sim* sim, const void* noise, double a0);

/* The same initial conditions from noise drawn on the device from `seed`:
 * element i of the Np^3 lattice (C order) is normal i of a counter-based
 * stream, Philox4x64-10 (Salmon et al., SC 2011) with key (seed, 0); block c
 * uses counter (c + 1, 0, 0, 0), its four words w become uniforms
 * u = (w >> 11) 2^-53 and, pairwise, normals by Box-Muller:
 * r = sqrt(-2 ln(1 - u0)), (r cos 2 pi u1, r sin 2 pi u1).  The noise is kept
 * for pm_init_ic_vjp as with pm_init_ic.  Errors as pm_init_ic. */
int pm_init_ic_seed(pm_sim* sim, uint64_t seed, double a0);

/* That noise alone, written to the device array noise_out [Np^3] (dtype).
 * Errors: PM_EINVAL (NULL noise_out). */
int pm_noise(pm_sim* sim, uint64_t seed, void* noise_out);

/* Reuse the arena for new physical parameters: cosmology, box, field of view
 * and source redshifts may change; Np, Nm, dtype, modes, npix and nsrc must
 * equal those of pm_create.  Rebuilds and uploads the float64 tables (the
 * PGD filter too, for the new box, when the correction is on) and clears
 * the state (pm_init_ic* must follow).  Waits for the stream.
 * Errors: PM_EINVAL (invalid or arena-changing parameters), PM_EDEVICE. */
int pm_reconfigure(pm_sim* sim, const pm_params* p, const lens_params* l);

/* One kick-drift-kick PM step from a0 to a1 (package design section: FastPM
 * kick and drift factors that keep linear displacement exact in every step):
 *   p += K(a0, ah; a0) f(x),  x += Dr(a0, a1; ah) p,  p += K(ah, a1; a1) f(x'),
 * with ah = (a0 + a1) / 2.  The force is cloud-in-cell painted, solved with
 * a Fourier Poisson kernel i k / k^2 and read back with cloud-in-cell.
 * The state must be at a0.  Errors: PM_ESTATE.  A non-finite position sets
 * the sticky device status that pm_sync reports. */
int pm_step(pm_sim* sim, double a0, double a1);

/* Born projection of the shell of step a0 -> a1 (convergence equation of the
 * notation section; lightcone and box replication of the design section):
 * every particle image with chi(a1) < chi <= chi(a0) adds
 *   w_s = 3/2 Om (H0/c)^2 V_p (chi_s - chi) / (chi_s chi a(chi) Omega_pix)
 * bilinearly at theta = r_perp / chi to map s (chi < chi_s), and every pixel
 * of map s gets the shell's mean term -3/2 Om (H0/c)^2 int q(chi)/a(chi) dchi.
 * `kappa` is a device array [nsrc][npix][npix], ACCUMULATED into; the caller
 * zeroes it before the first shell.  The state must be at a1.
 * Errors: PM_ESTATE, PM_EINVAL (NULL kappa). */
int lens_project(pm_sim* sim, double a0, double a1, void* kappa);

/* Sub-evolution ("interpolation" of the parameter table; the package-design
 * section's sub-evolution step), off by default.  When on, lens_project and
 * pm_run move every image before projecting it: the image keeps the shell of
 * its end-of-step depth chi_e, then follows its step's own drift,
 *   x(a) = x(a1) + (D(a) - D(a1)) / g_p(a_h) p_h,   a_h = (a0 + a1) / 2,
 * with p_h the momentum the step drifted with, to a = a(chi_e); its angles,
 * depth, a(chi) and weight are those of the moved image (the image may then
 * fall behind a source plane or off the map).  lens_project then needs the
 * state that pm_step(a0, a1) (or pm_run ending at a1) left, where
 * p_h = p - K2 f (else PM_ESTATE); lens_project_vjp and lens_project_jvp
 * differentiate it (see there).
 * on: 0 or 1.  Errors: PM_EINVAL (NULL sim). */
int pm_set_interpolation(pm_sim* sim, int32_t on);

/* PGD correction (the package-design section's first technique; the paper
 * names its parameters k_l, k_s, alpha0, mu and defers the operator to its
 * PGD reference), off by default.  When on, the positions that lens_project
 * and pm_run project at the end of step a0 -> a1 are
 *   x + S,  S = alpha0 a1^mu R(x, IFFT(O_l O_s i k delta_hat / k^2)),
 *   O_l = exp(-k_l^2 / k^2),  O_s = exp(-(k / k_s)^4),
 * the CIC readout at x of the force of x's own CIC density with that
 * filter; the run itself continues from the uncorrected state.  With
 * sub-evolution on as well, the corrected images are then moved.  Each
 * corrected projection costs the filtered force's axis-0, axis-1 and c2r
 * passes and one more readout: in pm_run the shift and the force share one
 * paint and the forward passes along axes 2 and 1 (lens_project after
 * pm_step paints and transforms once more).  k_l, k_s in h/Mpc; alpha0
 * dimensionless.  lens_project_vjp and lens_project_jvp refuse the mode
 * (PM_EINVAL).  The filter table, the displacement buffer and the spare mesh
 * are part of the arena of a handle created with PM_MODE_PGD.  on: 0 or 1.
 * Errors: PM_EINVAL (NULL sim, handle without PM_MODE_PGD, non-finite
 * parameter, k_l < 0 or k_s <= 0 with on = 1). */
int pm_set_pgd(pm_sim* sim, int32_t on, double alpha0, double mu, double k_l, double k_s);

/* Replica rotation (the package-design section: the box is rotated before it
 * is repeated, to avoid repeated structures along the line of sight), off by
 * default.  When on, the box replica with offsets (nx, ny, nz) is the box
 * under one of the 48 cube symmetries: index s = h % 48 of
 *   h = mix(seed ^ mix(u)),  u = (nx + 2^20) << 42 | (ny + 2^20) << 21 | (nz + 2^20),
 * mix being the 64-bit finalizer of SplitMix64; s takes the (s / 8)-th of
 * the six axis permutations in lexicographic order and reflects image axis j
 * (x -> L - x) when bit j of s % 8 is set; s = 0 is the identity.  Image
 * axis j of a particle is box axis perm(j).  Applies to lens_project,
 * pm_run and lens_project_vjp.  on: 0 or 1.  Errors: PM_EINVAL (NULL sim). */
int pm_set_replica_rotation(pm_sim* sim, int32_t on, uint64_t seed);

/* nsteps PM steps along the host array a_grid[0..nsteps] with the Born
 * projection of every step's shell into kappa (device [nsrc][npix][npix],
 * ACCUMULATED): the same results as pm_step(a_i, a_i+1) followed by
 * lens_project(a_i, a_i+1) for i = 0..nsteps-1, bit for bit, with less
 * memory traffic (each step's force readout also starts the next step:
 * half-kick, drift and sort keys).  The state must be at a_grid[0]; it ends
 * at a_grid[nsteps].  Errors: PM_EINVAL (NULL array, nsteps < 1),
 * PM_ESTATE. */
int pm_run(pm_sim* sim, const double* a_grid, int32_t nsteps, void* kappa);

/* Copy the state out, in lattice order: x [3][Np^3] in [0, L), p [3][Np^3]
 * (device arrays; either may be NULL).  *a_out receives the current scale
 * factor when a_out is non-NULL (a host pointer). */
int pm_get_state(pm_sim* sim, void* x_out, void* p_out, double* a_out);

/* Replace the state: x, p device arrays [3][Np^3] in lattice order, at scale
 * factor a.  Positions are taken modulo L; the force at x is recomputed.
 * Errors: PM_EINVAL. */
int pm_set_state(pm_sim* sim, const void* x, const void* p, double a);

/* Introspection of the last force evaluation (for tests): the painted
 * density rho (mean 1) [Nm^3], the three force meshes [3][Nm^3] in Mpc/h
 * (f = -grad inverse-Laplacian(rho - 1)), and the force at the particles
 * [3][Np^3] in lattice order.  Any pointer may be NULL. */
int pm_get_force(pm_sim* sim, void* rho_out, void* fmesh_out, void* acc_out);

/* Wait for the stream; return the sticky device status (PM_ENONFINITE if a
 * kernel saw a non-finite position), else PM_OK or PM_EDEVICE. */
int pm_sync(pm_sim* sim);

/* Kick and drift factors and growth used by the library, float64, for
 * tests: out[0] = D(a), out[1] = g_p(a), out[2] = chi(a) in Mpc/h. */
int pm_background(const pm_sim* sim, double a, double out[3]);

/* ---- reverse mode (vector-Jacobian products) ------------------------------
 * The paper makes the simulation differentiable by reverse-mode automatic
 * differentiation with respect to the initial Gaussian modes, Omega_m and
 * sigma_8, the cosmology dependence of scalar factors (kick/drift factors,
 * initial-condition growth and amplitude) being finite-differenced (design
 * section; appendix on cosmology derivatives).  These calls run that reverse
 * pass one shell / step at a time; the caller keeps checkpoints of (x, p)
 * with pm_get_state and restores them with pm_set_state.  Cotangent arrays
 * are device arrays [3][Np^3] of dtype in lattice order and Mpc/h units
 * (dL/dx, dL/dp).  cosmo_bar is a host array [2] = (dL/dOmega_m,
 * dL/dsigma_8), ACCUMULATED.  Omega_m derivatives of scalar factors are
 * central differences with step 1e-5; membership is held fixed: the distance
 * bounds of each shell, and which images lie in front of each source plane
 * (the lens weight vanishes there, so this changes no derivative).  With a
 * host cosmo_bar each call waits for its stream at the end (it reads reduced
 * scalars back).  cosmo_bar may be NULL: the call then adds its contribution
 * to an accumulator on the device, in stream order and without waiting, and
 * pm_vjp_cosmo_read returns the sum (a reverse pass then waits once).
 *
 * lens_project_vjp: state at a1.  x_bar += (d kappa_shell / dx)^T kappa_bar,
 * cosmo_bar[0] += kappa_bar . d kappa_shell / dOmega_m at fixed positions.
 * kappa_bar: device [nsrc][npix][npix].  With sub-evolution on, the shell
 * also depends on the step's drift momentum p_h = p - K2 f (the state's
 * force at a1): an image at end-of-step depth chi_e is projected at
 * r + dr p_h, dr = (D(a(chi_e)) - D(a1)) / g_p(a_h), so x_bar receives
 * g + e_z (d dr / d chi_e)(g . p_h) per image (g the splat's gradient at the
 * moved image), ph_bar (device [3][Np^3], lattice order, Mpc/h,
 * ACCUMULATED; required, else PM_EINVAL) receives dr g, and cosmo_bar[0]
 * the move's Omega_m derivative as well.  ph_bar belongs to pm_step_vjp of
 * the same step; it may be NULL when sub-evolution is off.  The PGD
 * correction has no reverse pass (PM_EINVAL).  Errors: PM_ESTATE, PM_EINVAL. */
int lens_project_vjp(pm_sim* sim, double a0, double a1, const void* kappa_bar, void* x_bar,
                     void* ph_bar, double cosmo_bar[2]);

/* pm_step_vjp: reverse of the step a0 -> a1.  The state must be at a1 (the
 * end of the step; the force there is that of pm_set_state or pm_step).  a2 >
 * a1 is the end of the following step, whose first half-kick uses the same
 * force, or a2 <= 0 when a0 -> a1 is the last step.  On entry x_bar, p_bar
 * hold the cotangents of (x, p) at a1 (after every later step and shell has
 * been reversed); on return they hold those at a0 (in place).  ph_bar
 * (read only, may be NULL) is the cotangent of this step's drift momentum
 * from lens_project_vjp(a0, a1) with sub-evolution: it joins p_bar at the
 * drift (the drift momentum does not pass through the force at a1).
 * Errors: PM_ESTATE, PM_EINVAL. */
int pm_step_vjp(pm_sim* sim, double a0, double a1, double a2, void* x_bar, void* p_bar,
                const void* ph_bar, double cosmo_bar[2]);

/* pm_init_ic_vjp: the state must be the initial conditions (restored with
 * pm_set_state at a0, after pm_init_ic was run on this handle with the same
 * noise); a1 is the end of the first step.  Reverses the first half-kick's
 * force and the Zel'dovich map: noise_bar (device [Np^3], WRITTEN) = dL/dnoise;
 * cosmo_bar += (dL/dOmega_m, dL/dsigma_8) of the initial conditions.
 * x_bar, p_bar are read only.  Errors: PM_ESTATE, PM_EINVAL. */
int pm_init_ic_vjp(pm_sim* sim, double a1, const void* x_bar, const void* p_bar, void* noise_bar,
                   double cosmo_bar[2]);

/* Checkpoints for the reverse pass, in the library's own particle order
 * (displacements, momenta, particle ids and the sort's block offsets): no
 * conversion to lattice order on save and no sort on load.  With
 * PM_MODE_CKPT_FORCE they also hold the force at the saved state.
 * pm_checkpoint_bytes: the size of one checkpoint of this handle (0 for a
 * NULL handle).  pm_checkpoint_save: copy the current state into buf (a
 * device buffer of that size, owned by the caller; asynchronous; with
 * PM_MODE_CKPT_FORCE the force is computed first if no call since the last
 * change of state has left it in the meshes).  pm_checkpoint_load: restore
 * a checkpoint made by a handle of the same shape and modes, at scale
 * factor a; the force there is copied from the checkpoint with
 * PM_MODE_CKPT_FORCE, else recomputed, as with pm_set_state (the same
 * values either way).  Errors: PM_EINVAL (NULL buffer, a <= 0), PM_ESTATE
 * (save without a state). */
size_t pm_checkpoint_bytes(const pm_sim* sim);
int pm_checkpoint_save(pm_sim* sim, void* buf);
int pm_checkpoint_load(pm_sim* sim, const void* buf, double a);

/* pm_vjp_cosmo_read: wait for the stream, add the device accumulator of the
 * calls above made with cosmo_bar = NULL to cosmo_bar (host [2]) and clear
 * it (it is also cleared by pm_create and pm_reconfigure).
 * Errors: PM_EINVAL (NULL pointer), PM_EDEVICE. */
int pm_vjp_cosmo_read(pm_sim* sim, double cosmo_bar[2]);

/* ---- forward mode (Jacobian-vector products) -------------------------------
 * The paper's automatic differentiation gives directional derivatives (Jvp)
 * as well as gradients, and its derivative checks (one perturbed
 * initial-condition pixel, sigma_8, Omega_m with single-mode initial
 * conditions) are Jvps against finite differences (section on validating
 * the derivatives).  These calls carry the tangent of the state along a
 * direction (noise_dot, Omega_m_dot, sigma8_dot) forward with the
 * simulation, one step / shell at a time, without checkpoints.  The
 * tangent (x_dot, p_dot and the force tangent f_dot at the current state)
 * is held by the library in its own particle order, and travels with the
 * particles through each step's sort; its 15 Np^3 values of dtype are part
 * of the arena of a handle created with PM_MODE_TANGENT (every call below
 * fails with PM_EINVAL on a handle without it).  pm_set_tangent and
 * pm_get_tangent exchange it with device arrays [3][Np^3] of dtype in
 * lattice order and Mpc/h.  Omega_m derivatives of scalar factors are the
 * central differences (step 1e-5) of the reverse mode, with the same fixed
 * shell partition and source membership; a tangent pass and a reverse pass
 * thus satisfy <kappa_bar, J v> = <J^T kappa_bar, v>.  The calls are
 * asynchronous on the simulation's stream.  Any call that changes the state
 * other than pm_step_jvp (pm_init_ic*, pm_step, pm_run, pm_set_state,
 * pm_reconfigure) drops the tangent.  Replica rotation and sub-evolution
 * have tangent passes; the PGD correction has none (PM_EINVAL from
 * lens_project_jvp).
 *
 * pm_init_ic_jvp: the state must be the initial conditions that pm_init_ic
 * (or pm_init_ic_seed) just made (no step, run or pm_set_state since, else
 * PM_ESTATE).  noise_dot: device [Np^3], the noise tangent.  Sets the tangent
 *   x_dot = D s_dot + Om_dot (dD/dOm) s,  p_dot = g_p s_dot + Om_dot (dg_p/dOm) s,
 *   s_dot = S(noise_dot + (s8_dot / s8) noise) + Om_dot dS/dOm(noise)
 * (S the Zel'dovich displacement map at D = 1), f_dot the force tangent at
 * the initial positions, and Omega_m_dot for the steps and shells to come.
 * Errors: PM_EINVAL (NULL array, non-finite scalar), PM_ESTATE. */
int pm_init_ic_jvp(pm_sim* sim, const void* noise_dot, double omega_m_dot, double sigma8_dot);

/* pm_set_tangent: set the tangent of the current state to (x_dot, p_dot)
 * (device [3][Np^3], lattice order, Mpc/h, read only) with Omega_m component
 * omega_m_dot; f_dot becomes the force tangent at the current positions: the
 * force meshes' gradient along x_dot read out at the particles, plus the
 * force of the tangent density (the cloud-in-cell paint differentiated
 * along x_dot) read out at the particles.
 * Errors: PM_EINVAL, PM_ESTATE (no state). */
int pm_set_tangent(pm_sim* sim, const void* x_dot, const void* p_dot, double omega_m_dot);

/* pm_get_tangent: copy the tangent out in lattice order (device [3][Np^3]
 * each; any may be NULL).  Errors: PM_ESTATE (no tangent). */
int pm_get_tangent(pm_sim* sim, void* x_dot, void* p_dot, void* f_dot);

/* pm_step_jvp: the step a0 -> a1 exactly as pm_step, and the tangent
 * carried across it:
 *   ph_dot = p_dot + K1 f_dot + Om_dot K1' f,  x_dot += Dr ph_dot + Om_dot Dr' (p + K1 f),
 *   f_dot = the force tangent at the new positions,  p_dot = ph_dot + K2 f_dot + Om_dot K2' f
 * (K1, Dr, K2 the step's kick, drift and kick factors, ' the Omega_m
 * difference).  The state must be at a0 with a tangent.
 * Errors: PM_EINVAL, PM_ESTATE. */
int pm_step_jvp(pm_sim* sim, double a0, double a1);

/* lens_project_jvp: state at a1, with a tangent.  kappa_dot (device
 * [nsrc][npix][npix], ACCUMULATED) += d kappa_shell along the tangent: per
 * image, (dw/dchi chi_dot + Om_dot dw/dOm) B + w (dB/dtheta . theta_dot)
 * with w the lens weight and B the bilinear weights, plus Om_dot times the
 * mean term's Omega_m difference.  With sub-evolution the image at end-of-
 * step depth chi_e is projected at r + dr p_h (see lens_project_vjp), and
 * its tangent is r_dot + (d dr / d chi_e) r_dot_z p_h + dr p_h_dot +
 * Om_dot (d dr / dOm) p_h with p_h_dot = p_dot - K2 f_dot - Om_dot K2' f.
 * Errors: PM_EINVAL (NULL array, PGD on), PM_ESTATE. */
int lens_project_jvp(pm_sim* sim, double a0, double a1, void* kappa_dot);

/* Per-kernel timing (tracing).  pm_profile(sim, 1) starts recording a pair
 * of HIP events around every kernel launch on the simulation's stream (the
 * events come from a pool created by this call, at most 8192 launches per
 * read); pm_profile(sim, 0) stops.  pm_profile_read waits for the stream and
 * writes, for up to max_kernels kernel names, the name (NUL-terminated, 32
 * bytes each, host array names[max_kernels][32]), the summed milliseconds and
 * the launch count since the last read, then resets the totals.  *n_out gets
 * the number of distinct names.  Any output array may be NULL. */
int pm_profile(pm_sim* sim, int enable);
/* Restricts the recording to launches of one kernel name (as pm_profile_read
 * reports it, e.g. "readout_kick_drift_key"); NULL or "" records every
 * launch again.  Each recorded launch adds two events to the stream, and
 * between kernels they cost time of their own, so a run timed as a whole
 * records only the kernel it reports.  The name is copied.  PM_EINVAL on a
 * NULL sim. */
int pm_profile_only(pm_sim* sim, const char* name);
int pm_profile_read(pm_sim* sim, int max_kernels, char* names, double* ms_total, long* counts,
                    int* n_out);

/* ---- serving ---------------------------------------------------------------
 * A request loop for many independent simulations on one GPU (the paper's
 * use case of fast simulations over many cosmologies): requests of any size
 * and cosmology are queued as they arrive, admitted in arrival order while
 * fewer than max_active run and the HBM footprint of their arenas
 * (pm_footprint plus the maps) fits hbm_budget, and run concurrently, each
 * on a stream of its own, their steps interleaved so that their kernels
 * overlap on the device (continuous batching).  Arenas of finished requests
 * stay allocated and are reused by later requests of the same shape, or
 * freed, least recently used first, when a new shape needs the memory.
 * max_active = 1 gives the plain form: one simulation at a time, first in
 * first out, with the same kernels.  Two host threads (admission, issue) run
 * inside the server; every call below is thread-safe. */
typedef struct pm_request {
    pm_params   p;         /* sizes, cosmology, dtype                          */
    lens_params l;         /* maps; z_src is copied at submission              */
    double      a_start;   /* initial conditions at a_start                    */
    double      a_end;     /* nsteps PM steps linear in a up to a_end          */
    int32_t     nsteps;
    uint64_t    seed;      /* white noise as in pm_init_ic_seed                */
} pm_request;

typedef struct pm_srv_stats {
    int64_t submitted, completed, failed;
    int32_t running, queued, peak_running;
    size_t  bytes_in_use, peak_bytes;  /* HBM held by arenas and maps        */
    double  now;                       /* server clock, seconds              */
} pm_srv_stats;

typedef struct pm_srv pm_srv;

/* Errors: PM_EINVAL (max_active < 1, zero budget), PM_ENOMEM. */
int pm_srv_create(size_t hbm_budget, int32_t max_active, pm_srv** out);

/* The same server with batched stepping when `batched` is 1: every running
 * request is a slot of the batch of its shape (pm_batch_*, capacity
 * max_active, each batch on a stream of its own), so same-shape requests
 * step together in one set of launches replayed from a HIP graph, up to two
 * batched steps in flight per batch; requests of other shapes run in their
 * own batches side by side.  batched = 0 is pm_srv_create.  A request's maps
 * are bit for bit those of the other forms.  Errors as pm_srv_create. */
int pm_srv_create_ex(size_t hbm_budget, int32_t max_active, int32_t batched, pm_srv** out);

/* Queue a request; *id_out identifies it.  The request's maps start at zero
 * and receive every shell of its steps.  Errors: PM_EINVAL (invalid
 * parameters or time range), PM_ENOMEM (footprint above the budget),
 * PM_ESTATE (server shutting down). */
int pm_srv_submit(pm_srv* s, const pm_request* r, int64_t* id_out);

/* Wait until the request has finished (successfully or not), at most
 * timeout_s seconds (< 0: no limit).  PM_OK when finished, PM_EAGAIN on
 * timeout, PM_EINVAL for an unknown id. */
int pm_srv_wait(pm_srv* s, int64_t id, double timeout_s);

/* For a finished request: copy its maps to the host buffer kappa_host
 * [nsrc][npix][npix] (dtype; may be NULL) and times[3] = (submitted,
 * admitted, finished) on the server clock, in seconds (may be NULL); then
 * forget the request.  Returns the request's status (PM_OK or the error that
 * ended it), PM_EAGAIN if it has not finished, PM_EINVAL for an unknown id. */
int pm_srv_result(pm_srv* s, int64_t id, void* kappa_host, double times[3]);

int pm_srv_stats_get(pm_srv* s, pm_srv_stats* out);

/* Drop queued requests, let running ones finish, free every arena. */
int pm_srv_destroy(pm_srv* s);

/* ---- batched stepping ---------------------------------------------------------
 * Many simulations of one shape (Np, Nm, dtype, npix, nsrc) stepped together,
 * each with its own arena, cosmology, box, field of view, time grid and maps
 * (the paper's use case of many fast simulations across cosmologies): one
 * launch per pass of the fused step serves every slot of the batch, so small
 * simulations fill the device together, and the launches are replayed from a
 * HIP graph captured at the first step (kernel nodes only).  Each slot's
 * arguments of every pass (its arena's pointers, the step's kick, drift and
 * kick factors, the shell's bounds, lens weights and mean terms) live in a
 * device parameter block that the batch rewrites before each replay (one
 * host-to-device copy on the batch's stream), so the captured graph replays
 * unchanged.  A slot's results are bit for bit those of pm_run on its handle
 * (float32; float64 to round-off).
 *
 * pm_batch_create: shape from p and l (their cosmology, box and geometry are
 * not used); capacity slots (1..1024); use_graph 0 launches the passes
 * directly instead of replaying the graph; hip_stream (NULL: a stream of the
 * batch's own) carries every batched launch.  Allocates the parameter block
 * (device) and its two pinned host copies.  Errors: PM_EINVAL, PM_ENOMEM,
 * PM_EDEVICE.
 * pm_batch_attach: sim (same shape, no sub-evolution, PGD or rotation) must
 * be at a_grid[0], its initial conditions made (pm_init_ic*); a_grid [0 ..
 * nsteps] (host, copied) is its time grid.  The batch's stream waits (an
 * event, not the host) for the work enqueued on the handle's stream so far,
 * then gets the first step's half-kick, drift and sort keys.  *slot_out (may be NULL) receives the slot.  Until
 * pm_batch_detach the handle belongs to the batch (no other call on it).
 * Errors: PM_EINVAL (NULL, shape or mode mismatch, attached already,
 * invalid grid), PM_ESTATE (state not at a_grid[0]), PM_EFULL.
 * pm_batch_lens: the maps (device [nsrc][npix][npix] of dtype, ACCUMULATED,
 * caller-owned) into which the shells of sim's coming steps are projected;
 * NULL projects none.  Errors: PM_EINVAL (not attached).
 * pm_batch_step: one fused step (pm_run's: sort, paint, the Born projection
 * of the step's shell, force, readout with the next step's half-kick, drift
 * and keys) of every attached slot with steps left, asynchronous on the
 * batch's stream; *running_out (may be NULL) receives the number of slots
 * with steps left after it.  A slot whose last step this was is at the end
 * of its time grid.
 * pm_batch_detach: frees sim's slot; the handle's stream waits (an event)
 * for the batch's work enqueued so far, so calls on the handle see its
 * results.  The handle then is at the end of its grid if it finished it,
 * else between two steps, where only pm_init_ic*, pm_set_state or
 * pm_checkpoint_load can continue it.  Errors: PM_EINVAL (not attached). */
typedef struct pm_batch pm_batch;
int pm_batch_create(const pm_params* p, const lens_params* l, int32_t capacity, int32_t use_graph,
                    void* hip_stream, pm_batch** out);
int pm_batch_attach(pm_batch* b, pm_sim* sim, const double* a_grid, int32_t nsteps,
                    int32_t* slot_out);
int pm_batch_lens(pm_batch* b, pm_sim* sim, void* kappa);
int pm_batch_step(pm_batch* b, int32_t* running_out);
int pm_batch_detach(pm_batch* b, pm_sim* sim);
int pm_batch_destroy(pm_batch* b);

/* ---- a run that allocates nothing -------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one whole
 * simulation, the same as pm_create, pm_init_ic(noise, a_grid[0]),
 * pm_run(a_grid, nsteps, kappa) and pm_destroy, with the arena placed in a
 * static device array of PM_NOALLOC_MAX_BYTES that the library holds on
 * every GPU it runs on until the process ends (a 64^3-particle, 128^3-mesh
 * float32 simulation needs 51 MiB).  No device memory is allocated or freed.
 * The call first waits for hip_stream (NULL = the default stream), whose
 * earlier calls may still use the array, uploads the host-side tables, and
 * returns with the run enqueued on hip_stream for the current device.  noise: device [Np^3] of dtype (read); kappa: device
 * [nsrc][npix][npix] of dtype, ACCUMULATED.  Every call on one GPU uses the
 * same array, so calls that overlap on one GPU (other streams, other host
 * threads) race; each call sets up everything it reads (the histogram, the
 * status word and the reverse-pass accumulator are cleared by kernels).
 * Errors: PM_EINVAL (invalid parameters, modes != 0, NULL pointer,
 * nsteps < 1, a0 as for pm_init_ic), PM_ETOOBIG (the arena, pm_footprint,
 * exceeds PM_NOALLOC_MAX_BYTES), PM_EDEVICE. */
#define PM_NOALLOC_MAX_BYTES (64u << 20)
int pm_run_noalloc(const pm_params* p, const lens_params* l, void* hip_stream, const void* noise,
                   const double* a_grid, int32_t nsteps, void* kappa);

const char* pm_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* MADLENS_H */
