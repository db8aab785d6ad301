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
#define PM_EFULL       -6   /* a batch has no free slot                      */

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
} pm_params;

typedef struct lens_params {
    int32_t       npix;     /* map pixels per side                           */
    double        fov_deg;  /* map side in degrees, (0, 22]                  */
    int32_t       nsrc;     /* number of source planes (maps), 1..16         */
    const double* z_src;    /* host array [nsrc] of source redshifts, copied */
} lens_params;

typedef struct pm_sim pm_sim;

/* Size rules: Nm and Np are multiples of 16 (Np >= 16), Nm / Np is 1 or 2,
 * Nm and Np have no prime factor other than 2 and 3 and are at most 1024;
 * 0 < Omega_m < 1; box > 0; 16 <= npix <= 8192.  Violations give PM_EINVAL. */

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
 * central differences with step 1e-5; shell membership (the distance bounds
 * of each shell) is held fixed.  Each call waits for its stream at the end
 * (it reads reduced scalars back).
 *
 * lens_project_vjp: state at a1.  x_bar += (d kappa_shell / dx)^T kappa_bar,
 * cosmo_bar[0] += kappa_bar . d kappa_shell / dOmega_m at fixed positions.
 * kappa_bar: device [nsrc][npix][npix].  Errors: PM_ESTATE, PM_EINVAL. */
int lens_project_vjp(pm_sim* sim, double a0, double a1, const void* kappa_bar, void* x_bar,
                     double cosmo_bar[2]);

/* pm_step_vjp: reverse of the step a0 -> a1.  The state must be at a1 (the
 * end of the step; the force there is that of pm_set_state or pm_step).  a2 >
 * a1 is the end of the following step, whose first half-kick uses the same
 * force, or a2 <= 0 when a0 -> a1 is the last step.  On entry x_bar, p_bar
 * hold the cotangents of (x, p) at a1 (after every later step and shell has
 * been reversed); on return they hold those at a0 (in place).
 * Errors: PM_ESTATE, PM_EINVAL. */
int pm_step_vjp(pm_sim* sim, double a0, double a1, double a2, void* x_bar, void* p_bar,
                double cosmo_bar[2]);

/* pm_init_ic_vjp: the state must be the initial conditions (restored with
 * pm_set_state at a0, after pm_init_ic was run on this handle with the same
 * noise); a1 is the end of the first step.  Reverses the first half-kick's
 * force and the Zel'dovich map: noise_bar (device [Np^3], WRITTEN) = dL/dnoise;
 * cosmo_bar += (dL/dOmega_m, dL/dsigma_8) of the initial conditions.
 * x_bar, p_bar are read only.  Errors: PM_ESTATE, PM_EINVAL. */
int pm_init_ic_vjp(pm_sim* sim, double a1, const void* x_bar, const void* p_bar, void* noise_bar,
                   double cosmo_bar[2]);

/* Per-kernel timing (tracing).  pm_profile(sim, 1) starts recording a pair
 * of HIP events around every kernel launch on the simulation's stream (the
 * events come from a pool created by this call, at most 8192 launches per
 * read); pm_profile(sim, 0) stops.  pm_profile_read waits for the stream and
 * writes, for up to max_kernels kernel names, the name (NUL-terminated, 32
 * bytes each, host array names[max_kernels][32]), the summed milliseconds and
 * the launch count since the last read, then resets the totals.  *n_out gets
 * the number of distinct names.  Any output array may be NULL. */
int pm_profile(pm_sim* sim, int enable);
int pm_profile_read(pm_sim* sim, int max_kernels, char* names, double* ms_total, long* counts,
                    int* n_out);

const char* pm_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* MADLENS_H */
