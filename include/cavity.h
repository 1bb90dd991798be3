/*
 * cavity.h - C ABI of the MI355X (gfx950) solver for time-harmonic electromagnetic
 * scattering from an open rectangular cavity in a perfectly conducting ground plane
 * (Chen, Jiang, Lai, Li, "A fast algorithm for the electromagnetic scattering from a
 * large rectangular cavity in three dimensions", arXiv 2008.01966).
 *
 * Problem statement (Section 2 of the paper): cavity [0,a] x [0,b] x [-c,0] below the
 * ground plane, aperture [0,a] x [0,b] at z = 0, walls and ground perfectly conducting,
 * non-magnetic medium with relative permittivity eps_r(z) piecewise constant in layers,
 * vacuum above the ground plane with wavenumber k, time convention e^{-i omega t}
 * (Im eps_r >= 0 is lossy).  Lengths are in any unit consistent with k (the paper's
 * examples use the wavelength, k = 2 pi).
 *
 * Method (Sections 3-6): the field components are expanded in the sine/cosine series
 * (E123F) with M = Nx-1, N = Ny-1 modes per axis; each mode's z-column is discretised by
 * second-order differences on Nz uniform intervals (h = c/Nz) and eliminated down to the
 * aperture (the LU relation r_JJ E_J + E_{J+1} = 0 and its layered form (uTT1)); the
 * transparent boundary condition (ENU1) couples the aperture modes through three
 * single-layer operators whose singular integrals are applied by FFT convolution with
 * the spectrum of the truncated kernel (Section 5); the reduced aperture system (EJ1) /
 * (uT1) is solved by preconditioned GMRES; the interior is recovered by
 * back-substitution (EInter) and the backscatter RCS is evaluated from the aperture
 * field (Section 7).
 *
 * Conventions shared by every entry point
 *  - Complex numbers are interleaved double pairs (cavity_c128).
 *  - "device" pointers are HIP device memory owned by the caller; they are written
 *    asynchronously on the plan's stream and valid after that stream is synchronised.
 *  - "host" pointers are ordinary host memory; calls taking host outputs synchronise
 *    the plan's stream before returning.
 *  - Every function returns a status (0 = CAVITY_OK).  On failure nothing is written to
 *    the outputs except where stated, and cavity_last_error() returns a message for the
 *    calling thread.
 *  - A plan is not thread-safe; distinct plans may be used from distinct threads/streams.
 *  - Device arrays of complex values passed in (E_out, aperture_out, a request's E_out)
 *    must be 16-byte aligned (as every hipMalloc or torch allocation is); a misaligned
 *    one gives CAVITY_EINVAL.
 *  - Field output layout E_out[3][Nz+1][Ny+1][Nx+1] (component, z-node, y-node, x-node;
 *    x fastest) on the nodes x = i1 a/Nx, y = i2 b/Ny, z = -c + j h.  At an interface
 *    node the normal component E3 is reported on the upper side.
 *  - Aperture vector layout (paper's Appendix A order): E1 on N1 = {0..M} x {1..N},
 *    then E2 on N2 = {1..M} x {0..N}, then E3 on N3 = {1..M} x {1..N}, each m-major;
 *    n_ap = (M+1)N + M(N+1) + MN entries.
 */
#ifndef CAVITY_H
#define CAVITY_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
  CAVITY_OK = 0,
  CAVITY_EINVAL = 1,     /* invalid argument (sizes, angles, NULL pointers, layer sums) */
  CAVITY_ENOMEM = 2,     /* plan footprint exceeds the HBM budget or allocation failed */
  CAVITY_ERESONANT = 3,  /* a z-elimination pivot vanished: discrete closed-cavity resonance */
  CAVITY_ENOCONV = 4,    /* GMRES did not reach the tolerance within max_iter */
  CAVITY_EDEVICE = 5,    /* HIP runtime error (detail in cavity_last_error) */
  CAVITY_ENOTIMPL = 6    /* option not implemented */
};

enum { CAVITY_FP64 = 0, CAVITY_MIXED = 1 };
enum { CAVITY_TBC_TRAP = 0, CAVITY_TBC_SPEC = 1 };
/* Evaluation of the kernel spectrum (cavity_opts.spectrum). */
enum { CAVITY_SPECTRUM_EXACT = 0, CAVITY_SPECTRUM_ASYMPTOTIC = 1 };
enum { CAVITY_TM = 0 /* theta-hat polarisation */, CAVITY_TE = 1 /* phi-hat */ };

typedef struct cavity_plan_s* cavity_plan; /* opaque; owns all of its device memory */

typedef struct {
  double re, im;
} cavity_c128;

/* Layer stack, bottom to top (Section 4 and its closing remark for more layers).
 * layer_nz[i] >= 1 intervals of layer i with sum equal to Nz; eps_r[i] its relative
 * permittivity.  Interfaces sit on the z-grid nodes.
 * layer_depth: NULL gives every layer the common step c / Nz (the paper's setting).
 * Otherwise layer i is layer_depth[i] > 0 thick (the thicknesses sum to c within 1e-12 c,
 * else CAVITY_EINVAL) with step layer_depth[i] / layer_nz[i], as Example 3 of Section 7
 * gives its layers different interval counts.  The interface conditions of Section 4
 * are then discretised with each one-sided difference over its own layer's step, and the
 * aperture rows (Section 5) use the top layer's step.  The request server (below) builds
 * its plans with the common step. */
typedef struct {
  int n_layers;
  const int* layer_nz;        /* host, n_layers entries */
  const cavity_c128* eps_r;   /* host, n_layers entries */
  const double* layer_depth;  /* host, n_layers entries, or NULL */
} cavity_eps;

/* Solver options; cavity_opts_default() fills the defaults listed here. */
typedef struct {
  int precision;        /* CAVITY_FP64 (default), or CAVITY_MIXED: the three TBC convolutions
                           inside the GMRES iterations run in single precision (transforms,
                           spectrum, workspaces); each restart recomputes the residual with the
                           double-precision operator (iterative refinement), so tol applies to
                           the double-precision system.  Elimination, profiles, right-hand
                           sides, Krylov vectors, synthesis and RCS stay double. */
  int tbc_oversample;   /* s >= 1: TBC quadrature grid has s*Nx x s*Ny intervals (default 1) */
  double tol;           /* relative residual of the aperture system (default 1e-12) */
  int max_iter;         /* total GMRES iterations per right-hand side (default 400) */
  int restart;          /* GMRES restart length, 1..200 (default 60) */
  size_t hbm_budget;    /* bytes the plan may allocate; 0 = 90 % of free device memory */
  void* stream;         /* hipStream_t for all work of the plan; NULL = default stream */
  int batch;            /* right-hand sides iterated together in lockstep, 1..64 (default 8) */
  int direct;           /* direct solve (the paper's Steps 1 and 3, Section 6: the aperture
                           matrix assembled from the operator and inverted once per plan by
                           Gauss-Jordan elimination with partial pivoting, 2 (3 Nx Ny)^2 x 16
                           bytes while it is built, half that kept; each right-hand side is
                           then one product with the inverse plus a residual check):
                           0 = automatic (default): used when 3 Nx Ny <= 2048 and a call solves
                           at least 32 right-hand sides, and for every call once the inverse
                           exists; 1 = always (3 Nx Ny <= 4096, else CAVITY_EINVAL at plan
                           creation); -1 = never (GMRES only) */
  int tbc_operator;     /* discrete TBC (Section 5): CAVITY_TBC_TRAP (default) samples the
                           trial functions on the trapezoid grid and convolves by FFT;
                           CAVITY_TBC_SPEC uses their exact Fourier transforms on the same
                           kernel-spectrum lattice (second-order accurate in the lattice
                           size, about ten times closer to the exact Galerkin integrals),
                           applied as four dense complex products per family in double
                           precision in both precision modes; its work grows as
                           P1 P2 (M + N) per family, so it suits small and mid-size cavities */
  int spectrum;         /* kernel spectrum (Section 5.2): CAVITY_SPECTRUM_EXACT (default)
                           integrates the radial J0 integral by quadrature at every lattice
                           frequency rho; CAVITY_SPECTRUM_ASYMPTOTIC uses the paper's Case 2
                           (two-term Hankel expansion of J0, Fresnel tails) where
                           (rho - k) R >= 100, with an error below about 1e-8 of the
                           spectrum's largest value, and the quadrature elsewhere */
} cavity_opts;

/* Plan description and the statistics of its last solve. */
typedef struct {
  int M, N, Nz;
  int P1, P2;                  /* FFT box of the TBC convolution */
  long long n_ap;              /* aperture unknowns */
  long long unknowns;          /* n_ap * Nz: unknowns per right-hand side */
  size_t device_bytes;         /* device memory held by the plan */
  double min_pivot;            /* smallest |pivot| met in the z-elimination */
  int last_iterations;         /* GMRES iterations of the last solve */
  double last_rel_residual;    /* true relative residual of the last solve */
  double ms_spectrum, ms_elimination, ms_preconditioner; /* plan phases (device time) */
  double ms_rhs, ms_krylov, ms_synthesis;                /* last solve phases */
  int lds_budget;              /* LDS bytes per block the TBC FFT kernels are sized for
                                  (chosen by timing at the first plan of a shape; 0 = the
                                  default 40000 or CAVITY_LDS_BUDGET) */
  int last_direct;             /* 1 when the last solve call used the direct solve
                                  (last_iterations is then 0) */
  double ms_factor;            /* device time of assembling and inverting the aperture
                                  matrix for the direct solve (0 until it is built) */
  int tbc_rows_in_place;       /* 1 when the TBC row passes run their transforms in place
                                  in LDS (one buffer per transform), 0 for the two-buffer
                                  form; chosen by timing with lds_budget */
} cavity_info;

int cavity_opts_default(cavity_opts* opts);

/* Build a plan: validates arguments, derives sizes, allocates device memory, computes
 * the truncated-kernel spectrum (Section 5), runs the per-mode z-elimination (Sections
 * 3-4) and the block preconditioner.  a, b, c, k > 0; Nx, Ny >= 2; Nz >= 1; eps may be
 * NULL (vacuum).  opts may be NULL.  The sine/cosine transforms run as FFTs of lengths
 * 2 Nx, 2 Ny, 2 s Nx and 2 s Ny built from radices with the prime factors 2, 3, 5, 7, 11
 * and 13; a length with another prime factor gives CAVITY_ENOTIMPL.
 * Errors: CAVITY_EINVAL, CAVITY_ENOMEM, CAVITY_ERESONANT, CAVITY_ENOTIMPL, CAVITY_EDEVICE. */
int cavity_plan_create(double a, double b, double c, int Nx, int Ny, int Nz,
                       const cavity_eps* eps, double k, const cavity_opts* opts,
                       cavity_plan* out);

/* Solve for one plane wave (Section 7): direction angles theta in [0, pi/2], phi any,
 * pol CAVITY_TM or CAVITY_TE.  Writes the field on all nodes to E_out (device, caller
 * owned, 3*(Nz+1)*(Ny+1)*(Nx+1) entries) unless E_out is NULL; keeps the aperture
 * solution in the plan as right-hand side 0 for cavity_rcs / cavity_aperture.
 * Errors: CAVITY_EINVAL, CAVITY_ENOCONV (E_out still written with the last iterate),
 * CAVITY_EDEVICE. */
int cavity_solve(cavity_plan plan, double theta, double phi, int pol, cavity_c128* E_out);

/* Solve nrhs plane waves (host arrays theta, phi, pol) on the plan's stream, opts.batch
 * of them at a time iterating together (every kernel launch serves the whole group).  The
 * paper computes the singular-integral data once per geometry and reuses it for every
 * incidence (Section 7, Example 1; Steps 1-3 of Section 6): here the plan is that data,
 * and each right-hand side is one reduced aperture system (EJ1) / (uT1) with the source
 * g of (ENUC1) for its wave.  E_out (device) holds nrhs consecutive fields or is NULL;
 * aperture_out (device) holds nrhs consecutive aperture vectors of n_ap entries or is
 * NULL.  The plan keeps the aperture solutions of this call only (indices 0..nrhs-1) for
 * cavity_rcs; those of earlier calls are forgotten.
 * Errors: CAVITY_EINVAL (nrhs < 1, NULL arrays, angles as for cavity_solve),
 * CAVITY_ENOCONV (every field still written), CAVITY_ENOMEM, CAVITY_EDEVICE. */
int cavity_solve_batch(cavity_plan plan, int nrhs, const double* theta, const double* phi,
                       const int* pol, cavity_c128* E_out, cavity_c128* aperture_out);

/* Solve n small cavities together, one plane wave each: plans[r] (distinct plans) at
 * (theta[r], phi[r], pol[r]).  The transparent boundary operator of Section 5 depends only
 * on the aperture, so cavities that share it (equal a, b, Nx, Ny, k, tbc_oversample and
 * spectrum) but differ in depth, z-grid or layers (their own columns of Sections 3-4, their
 * own aperture step h) iterate as one lockstep group: every kernel launch of the Krylov
 * solve serves all n of them, each right-hand side with its own cavity's local blocks and
 * preconditioner.  The plans must also share precision, tol, restart and max_iter, use the
 * trapezoid operator (else CAVITY_ENOTIMPL) and not be used by another thread meanwhile;
 * the work runs on plans[0]'s stream (workspace of plans[0] sized for n right-hand sides),
 * and the call synchronises it before returning.  Afterwards every plan keeps its own
 * solution as right-hand side 0 (cavity_rcs, cavity_aperture) and E_out[r] (device,
 * [3][Nz+1][Ny+1][Nx+1] of plans[r]) holds its field unless E_out or E_out[r] is NULL.
 * Each result equals that of cavity_solve on the plan alone up to rounding.
 * Errors: CAVITY_EINVAL (n outside 1..64, NULL or repeated plans, plans that do not share
 * the aperture or options, angles), CAVITY_ENOTIMPL, CAVITY_ENOCONV, CAVITY_ENOMEM,
 * CAVITY_EDEVICE. */
int cavity_solve_group(int n, const cavity_plan* plans, const double* theta, const double* phi,
                       const int* pol, cavity_c128* const* E_out);

/* Radar cross section (units of length squared) of stored solution rhs_index at n_obs
 * observation directions (host arrays); sigma (host) receives {sigma_theta, sigma_phi}
 * per direction.  Backscatter: observation direction equal to the incidence angles, the
 * theta-theta and phi-phi RCS of Section 7.  The far field is radiated by the aperture's
 * tangential field with image doubling (the representation (EGa2) of Section 2): with
 * E^l(u) the aperture transform of E_l at u = k (sin t cos f, sin t sin f) and
 * L = (-E^2, E^1, 0), sigma_theta = (k^2/pi) |phi^.L|^2, sigma_phi = (k^2/pi) |theta^.L|^2.
 * Errors: CAVITY_EINVAL (no such solution), CAVITY_EDEVICE. */
int cavity_rcs(cavity_plan plan, int rhs_index, int n_obs, const double* theta_o,
               const double* phi_o, double* sigma);

/* The RCS above (Section 7) for n (solution, direction) pairs at once, e.g. the
 * backscatter of every incidence of a sweep such as the paper's RCS-versus-theta curves:
 * pair i is stored solution rhs_index[i] seen from (theta_o[i],
 * phi_o[i]); sigma[2 i], sigma[2 i + 1] = {sigma_theta, sigma_phi}.  One kernel launch and
 * one device-to-host copy for all pairs (cavity_rcs with n_obs directions is this call
 * with a repeated index; results are identical).  The plan keeps a device buffer of at
 * most 2.1 KB per pair of its largest call.  Errors: CAVITY_EINVAL, CAVITY_EDEVICE. */
int cavity_rcs_many(cavity_plan plan, int n, const int* rhs_index, const double* theta_o,
                    const double* phi_o, double* sigma);

/* cavity_rcs_many for callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same pairs, the same
 * aperture-transform kernel and the same results up to rounding (the block sums are added
 * on the device in the same order), with no allocation at all.  Its queries, partial sums
 * and results use a fixed 4 MiB device array of the library, one per device, held until the
 * process ends: the pairs must fit in it, n (60 + 32 B) bytes plus alignment with
 * B = min(64, ceil((M+1)(N+1)/256)) blocks per pair (at least 1900 pairs for any plan),
 * else CAVITY_EINVAL.  All calls on one device share that array: calls that overlap on a
 * device race, so the caller serialises them.  sigma (host) as for cavity_rcs_many; the call
 * synchronises the plan's stream.  Errors: CAVITY_EINVAL, CAVITY_EDEVICE. */
int cavity_rcs_many_noalloc(cavity_plan plan, int n, const int* rhs_index,
                            const double* theta_o, const double* phi_o, double* sigma);

/* Copy stored aperture solution rhs_index to host memory (n_ap entries, paper order). */
int cavity_aperture(cavity_plan plan, int rhs_index, cavity_c128* out_host);

/* Device bytes cavity_plan_create would allocate for these arguments with one right-hand
 * side in flight (plan data, solve workspace, one solution), without allocating anything.
 * Same validation and errors as cavity_plan_create (CAVITY_EINVAL). */
int cavity_plan_footprint(double a, double b, double c, int Nx, int Ny, int Nz,
                          const cavity_eps* eps, double k, const cavity_opts* opts,
                          size_t* bytes);

/* Sizes of the plan (M, N, the aperture unknowns 3MN + M + N of Section 6's complexity
 * table, the FFT box of Section 5) and the device times of its phases, which mirror the
 * paper's T_singular (spectrum), T_assemble (elimination, preconditioner) and T_solve
 * (Krylov, synthesis) of Section 7.  Errors: CAVITY_EINVAL (NULL arguments). */
int cavity_plan_info(cavity_plan plan, cavity_info* out);
void cavity_plan_destroy(cavity_plan plan);
const char* cavity_status_string(int status);
const char* cavity_last_error(void);

/* ---- Request server (serving many cavities) ---------------------------------------
 * A request is one cavity (geometry, grid, layers, k) and one incidence; its result is
 * the field on all nodes (the E_out of cavity_solve) and the backscatter RCS.  The server
 * runs requests on `streams` worker threads, each with its own HIP stream on the device
 * that was current when the server was created, so requests overlap on the GPU.
 * Admission: a free worker takes the oldest queued request whose device footprint
 * (cavity_plan_footprint, plus its field when the server holds it) fits in what the budget
 * leaves, so a large request at the head does not hold back smaller ones that fit; once the
 * head has been passed over for 25 ms, nothing else is admitted until it starts.  Requests
 * larger than the whole budget fail with CAVITY_ENOMEM.  The kernel spectrum and operator
 * diagonal of an aperture are cached across plans (Section 5 quantities depend on a, b, k,
 * Nx, Ny only), and the whole plan of a finished request (spectrum, per-mode elimination of
 * Sections 3-4, preconditioner, workspaces) stays resident, charged to the budget, for a
 * later request on the same cavity, which then skips plan creation; resident plans are
 * dropped least recently used first when admission needs their memory or their total
 * exceeds plan_cache_bytes.  Queued requests on cavities that share the aperture of the
 * request a worker takes (a, b, Nx, Ny, k), without a resident plan, are taken with it, up
 * to 8, as far as the budget allows, and solved as one lockstep group (cavity_solve_group).
 * Results are independent of the mix, of plan reuse and of grouping: a
 * request computes exactly what cavity_plan_create + cavity_solve + cavity_rcs compute for
 * it alone.  All functions are thread-safe. */
typedef struct cavity_server_s* cavity_server;

typedef struct {
  int streams;          /* concurrent requests (worker threads / HIP streams), 1..16 (default 4) */
  size_t hbm_budget;    /* device bytes all admitted requests hold together; 0 = 80 % of the
                           free device memory at creation */
  int precision;        /* CAVITY_FP64 or CAVITY_MIXED (default) */
  double tol;           /* GMRES tolerance (default 1e-12) */
  size_t plan_cache_bytes; /* most device bytes of resident plans kept for repeated cavities
                              (inside the budget); (size_t)-1, the default, = 25 % of the
                              budget; 0 = no plan reuse */
} cavity_server_opts;

typedef struct {
  double a, b, c;
  int Nx, Ny, Nz;
  int n_layers;                 /* 0 = vacuum, else layer_nz / eps_r as in cavity_eps */
  const int* layer_nz;          /* host, copied at submission */
  const cavity_c128* eps_r;     /* host, copied at submission */
  double k, theta, phi;
  int pol;
  cavity_c128* E_out;           /* device, caller-owned, [3][Nz+1][Ny+1][Nx+1]: complete when
                                   cavity_server_wait returns; NULL: the field is computed into
                                   a temporary server buffer (counted in the budget) */
} cavity_request;

typedef struct {
  int status;                   /* CAVITY_OK or the request's error */
  double sigma[2];              /* backscatter {sigma_theta, sigma_phi} */
  int iterations;
  double rel_residual;
  long long unknowns;           /* n_ap * Nz */
  size_t device_bytes;          /* bytes the request held while running */
  double t_submit_ms, t_start_ms, t_done_ms;   /* server clock: ms since creation */
  int plan_reused;              /* 1 when the request ran on a resident plan of an earlier
                                   request on the same cavity */
  int group_size;               /* requests solved together with this one in one lockstep
                                   group (cavity_solve_group), 1 when alone */
} cavity_result;

int cavity_server_opts_default(cavity_server_opts* opts);
/* Errors: CAVITY_EINVAL (opts out of range), CAVITY_EDEVICE. */
int cavity_server_create(const cavity_server_opts* opts, cavity_server* out);
/* Queue a request; *ticket identifies it.  Errors: CAVITY_EINVAL (argument validation as
 * cavity_plan_create, or a server being destroyed). */
int cavity_server_submit(cavity_server server, const cavity_request* req, long long* ticket);
/* Block until request `ticket` has completed and copy its result (the request's own
 * status is in out->status; the call returns CAVITY_EINVAL for an unknown ticket). */
int cavity_server_wait(cavity_server server, long long ticket, cavity_result* out);
/* Forget a completed request (its ticket becomes unknown). */
int cavity_server_release(cavity_server server, long long ticket);
/* Milliseconds on the server clock (steady clock since creation). */
double cavity_server_now_ms(cavity_server server);
/* Finish every queued request, stop the workers and free everything. */
void cavity_server_destroy(cavity_server server);

/* ---- Kernel timing probe (benchmarking) ------------------------------------------
 * Process-wide.  cavity_probe_kernel(which, capacity) starts watching one kernel
 * (CAVITY_K_*; which < 0 stops and frees the probe): each of its next `capacity`
 * launches, from any plan, is bracketed by HIP events on its launch stream and tagged
 * with its algorithmic byte count (the data the launch must read and write).
 * cavity_probe_read() waits for the recorded events and returns the number of launches,
 * their summed device time in ms and their summed algorithmic bytes.  Errors:
 * CAVITY_EINVAL, CAVITY_ENOMEM (more launches than capacity), CAVITY_EDEVICE. */
enum {
  CAVITY_K_SPECTRUM = 0, CAVITY_K_ELIMINATION = 1, CAVITY_K_TBC_ROWS_FWD = 2,
  CAVITY_K_TBC_COLS = 3, CAVITY_K_TBC_ROWS_BWD = 4, CAVITY_K_EPILOGUE = 5,
  CAVITY_K_SYNTH_ROWS = 6, CAVITY_K_SYNTH_COLS = 7,
  /* the three TBC passes in single precision (CAVITY_MIXED inner iterations) */
  CAVITY_K_TBC_ROWS_FWD_F32 = 8, CAVITY_K_TBC_COLS_F32 = 9, CAVITY_K_TBC_ROWS_BWD_F32 = 10
};
int cavity_probe_kernel(int which, int capacity);
int cavity_probe_read(int* launches, double* total_ms, double* total_bytes);

/* ---- Inspection of individual steps (host in, host out; for parity testing) ------
 * Mode-grid arrays are (M+1) x (N+1), m-major; entries outside a component's mode set
 * are zero. */

/* Schur data of the elimination: rho_d, T (tau_1 = mu_m T, tau_2 = nu_n T), rho_n. */
int cavity_debug_columns(cavity_plan plan, cavity_c128* rho_d, cavity_c128* T,
                         cavity_c128* rho_n);
/* Profiles at nodes 0..Nz: pi_d, theta_d (zero when homogeneous), pi_n; each
 * (Nz+1) x (M+1) x (N+1). */
int cavity_debug_profiles(cavity_plan plan, cavity_c128* pi_d, cavity_c128* theta_d,
                          cavity_c128* pi_n);
/* Kernel spectrum K^ on the P1 x P2 FFT lattice (FFT index order, unscaled). */
int cavity_debug_spectrum(cavity_plan plan, cavity_c128* khat);
/* Single-layer operator family f (0 = cos-sin, 1 = sin-cos, 2 = cos-cos) applied to a
 * coefficient grid. */
int cavity_debug_tbc(cavity_plan plan, int family, const cavity_c128* in, cavity_c128* out);
/* Reduced aperture operator (no preconditioner) on a padded 3 x (M+1) x (N+1) vector. */
int cavity_debug_operator(cavity_plan plan, const cavity_c128* in, cavity_c128* out);
/* Right-hand side grids g1, g2 of one incidence. */
int cavity_debug_rhs(cavity_plan plan, double theta, double phi, int pol, cavity_c128* g1,
                     cavity_c128* g2);
/* Stage radices the transform planner gives a plan with the six transform lengths len[6]
 * (the extension transforms 2 s Nx and 2 s Ny, the box transforms P1 and P2, the output
 * transforms 2 Nx and 2 Ny; Section 5 and the node sums of EInter are evaluated by these
 * FFTs).  radices: caller-owned host array [6][20], each length's stage radices in
 * execution order, unused entries 0; nst: [6] stage counts, 0 for a length that has no
 * factorisation into the supported radices.  Host only: no device is touched.  Errors:
 * CAVITY_EINVAL (NULL argument, a length below 1 or above 2^20). */
int cavity_debug_fft_plans(const int* len, int* radices, int* nst);

#ifdef __cplusplus
}
#endif

#endif /* CAVITY_H */
