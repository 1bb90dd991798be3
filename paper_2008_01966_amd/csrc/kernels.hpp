// Host-visible launchers of the cavity kernels and the parameter blocks they take.
// Every launcher enqueues work on the given stream and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"
#include "fft.hpp"

namespace cav {

// Sizes and scalars of one plan, passed by value to the kernels.
struct Geo {
  int M, N, Nz, NM;     // modes per axis, z-intervals, (M+1)(N+1)
  int nq1, nq2;         // TBC quadrature intervals per axis (s*Nx, s*Ny)
  int P1, P2;           // FFT box of the TBC convolution
  int ldx;              // row stride of the TBC workspaces X, Y: P2 rounded up to 16 entries,
                        // so every row starts on a 128-byte line
  int nx, ny;           // output grid intervals (Nx, Ny)
  double a, b, h, k;
  double hq1, hq2;
  double pa, pb, iab;   // pi / a, pi / b, 1 / (a b): mode wavenumbers mu = m pa, nu = n pb
                        // without a division per mode in the hot loops
  int lds_budget;       // LDS bytes per block the TBC FFT kernels size their batch for (0: default)
  int rows_ip;          // TBC row passes: 1 = in-place transforms allowed, 0 = ping-pong form
};

// An FFT length with its device stage twiddle tables (double and single precision; layout in
// FftPlan).
struct Fft {
  FftPlan p;
  const zd* tw;
  const zf* twf;
};
template <typename T>
__device__ inline const cx<T>* twiddles(const Fft& f);
template <>
__device__ inline const zd* twiddles<double>(const Fft& f) { return f.tw; }
template <>
__device__ inline const zf* twiddles<float>(const Fft& f) { return f.twf; }

// Largest radix compiled into the FFT kernels (the planner's limit).  Each FFT kernel also
// has a form compiled with radices up to 8 only: about half the registers, so more waves
// per SIMD; a plan uses it when all its transform lengths factor into radices up to 8.
constexpr int kMaxRadix = 16;
constexpr int kSmallRadix = 8;

// The transforms one plan needs.
struct Trig {
  Fft ext1, ext2;   // length 2*nq1, 2*nq2: sine/cosine transforms on the TBC grid
  Fft box1, box2;   // length P1, P2: the zero-padded convolution
  Fft out1, out2;   // length 2*Nx, 2*Ny: sine/cosine transforms on the output grid
  int maxr;         // largest radix of the six plans (kSmallRadix or kMaxRadix kernels)
};

// Layer description on the z-grid for the elimination kernel.
struct Layers {
  const int* node_code;   // per node j = 0..Nz: >= 0 interior of that layer, -(s+1) interface s
  const zd* kappa2;       // per layer: k^2 eps_r
  const zd* ratio;        // per interface: eps_upper / eps_lower
  const double* h;        // per layer: grid step (interface s lies between layers s, s+1)
  int layered;            // 1 when there is at least one interface
};

// Plane-wave data of one right-hand side, set up on the host (Section 7 incidence), and the
// aperture step h of its cavity (the one-sided difference of the aperture rows).
struct Wave {
  double alpha1, alpha2, beta;
  double p1, p2, p3;
  double h;
};

// Column data (Sections 3-4) of the cavities one lockstep group solves: right-hand side r
// uses rho_d, T, rho_n (NM each) and the 3x3 block preconditioner pinv (9 NM) at offset
// r * cs from these pointers (cs = 0: one cavity for the whole group), and the aperture
// step hs[r] (hs = nullptr: Geo::h).
struct Cols {
  const zd* rho_d;
  const zd* T;
  const zd* rho_n;
  const zd* pinv;
  long long cs;
  const double* hs;
};

// One aperture-transform evaluation behind an RCS value: stored solution rhs at the
// transform point (u1, u2) = k sin(theta_o) (cos(phi_o), sin(phi_o)).
struct RcsQuery {
  int rhs;
  double u1, u2;
};

// ---- timing probe ----------------------------------------------------------------
// Kernel identifiers for the benchmark probe (cavity_probe_* in the C ABI).
enum KernelId {
  K_SPECTRUM = 0, K_ELIMINATION = 1, K_TBC_ROWS_FWD = 2, K_TBC_COLS = 3, K_TBC_ROWS_BWD = 4,
  K_EPILOGUE = 5, K_SYNTH_ROWS = 6, K_SYNTH_COLS = 7, K_TBC_ROWS_FWD_F32 = 8,
  K_TBC_COLS_F32 = 9, K_TBC_ROWS_BWD_F32 = 10, K_COUNT = 11
};
// While the probe watches kernel `id`, these bracket its launches with HIP events on the
// launch stream and record the launch's algorithmic bytes; otherwise they do nothing.
void probe_begin(int id, hipStream_t st);
bool g_probe_active();   // a kernel is being watched
void probe_end(int id, hipStream_t st, double bytes);

// ---- plan-time kernels ------------------------------------------------------------
// method 0: quadrature everywhere; 1: the asymptotic (Case 2) form where (rho - k) R >= 100
hipError_t launch_spectrum(const Geo& g, double R, double scale, int method, zd* khat,
                           hipStream_t st);
hipError_t launch_elimination(const Geo& g, const Layers& ly, zd* rho_d, zd* T, zd* rho_n,
                              zd* pi_d, zd* theta_d, zd* pi_n, double* pivmin,
                              hipStream_t st);
hipError_t launch_basis_power(const Geo& g, const Trig& t, double* pw1, double* pw2,
                              hipStream_t st);
hipError_t launch_diag_contract(const Geo& g, const zd* khat, const double* pw1,
                                const double* pw2, zd* tmp, zd* diag, hipStream_t st);
hipError_t launch_min(const double* v, long long n, double* out, hipStream_t st);
hipError_t launch_precond_build(const Geo& g, const zd* rho_d, const zd* T, const zd* rho_n,
                                const zd* diag, zd* pinv, hipStream_t st);

// ---- solve-time kernels -----------------------------------------------------------
// Device state of GMRES for nb right-hand sides iterating in lockstep (restart length R):
// H[r][j][0..R] Hessenberg columns rotated in place into R, rotations cs/sn[r][0..R-1],
// rotated right-hand side g[r][0..R], solution weights y[r][0..R-1], norms nrm2[r],
// |b_r| in bnorm[r], active[r] (still iterating in this cycle), incycle[r] (started this
// cycle), jcount[r] (columns built in this cycle).
struct Krylov {
  zd *H, *cs, *sn, *g, *y;
  double *nrm2, *bnorm, *thr;   // thr[r]: a cycle of rhs r stops once |g_{j+1}| <= thr[r]
  double* relres;               // relative residual of rhs r at the start of the last cycle
  int *active, *incycle, *jcount;
  int* iters;                   // iterations done by rhs r over all cycles
  int* hflags;                  // host-mapped: after step j, hflags[j * nbh + r] = active[r]
  double* hratio;               // host-mapped: after step j, |g_{j+1}| / thr[r] of rhs r
  int nbh;
  int restart;
  double tol;
};

hipError_t launch_rhs(const Geo& g, const Wave* waves, int nb, zd* b, hipStream_t st);
// y_r = A (P^{-1} v_r) when precond != 0, else y_r = A v_r, for r < nb with active[r] (or all
// when active is null).  v_r = v + r vs, y_r = y + r ys.  X, Y: nb x 3 x (M+1) x P2 and
// S: nb x 3 x NM workspaces.
// Trial-function transforms of the spectral TBC operator (D_spec): F1 [P1][M+1] for the cos
// and sin bases along x, F2 [P2][N+1] along y.
struct SpecMats {
  const zd *f1c, *f1s, *f2c, *f2s;
};
hipError_t launch_spec_passes(const Geo& g, const SpecMats& sm, const zd* khat, const zd* pinv,
                              int precond, int fam_fixed, int nb, const zd* v, long long vs,
                              zd* X, zd* Y, zd* U, zd* S, const int* active, hipStream_t st);
hipError_t launch_operator_spec(const Geo& g, const SpecMats& sm, const zd* khat, const Cols& c,
                                int precond, int nb, const zd* v, long long vs, zd* X, zd* Y,
                                zd* U, zd* S,
                                zd* y, long long ys, const int* active, hipStream_t st);

hipError_t launch_operator(const Geo& g, const Trig& t, const zd* khat, const Cols& c,
                           int precond, int nb, const zd* v, long long vs, zd* X, zd* Y, zd* S,
                           zd* y, long long ys,
                           const int* active, hipStream_t st);
// The same operator with the three single-layer convolutions in single precision
// (spectrum khat_f, workspaces Xf, Yf of the same element count as X, Y; S holds the TBC
// results in single precision); y and the local terms stay double.
hipError_t launch_operator_f32(const Geo& g, const Trig& t, const zf* khat_f, const Cols& c,
                               int precond, int nb, const zd* v, long long vs, zf* Xf, zf* Yf,
                               zd* S, zd* y,
                               long long ys, const int* active, hipStream_t st);
// ... on a vector v stored in single precision.
hipError_t launch_operator_f32(const Geo& g, const Trig& t, const zf* khat_f, const Cols& c,
                               int precond, int nb, const zf* v, long long vs, zf* Xf, zf* Yf,
                               zd* S, zd* y, long long ys, const int* active, hipStream_t st);
// The operator on v (P^{-1} applied to it first when precond) into y, its epilogue fused
// with the first Gram-Schmidt dot products against nv <= 16 basis vectors V (basis vector
// t of right-hand side r at V + t ldj + r 3 NM): out[r * ostride + t] = sum conj(V_t,r) y_r,
// from nblk per-block partial sums in `partial` (nb * nvmax * nblk entries).  The input
// and the output may be stored in single precision (last two overloads).
hipError_t launch_operator_dots(const Geo& g, const Trig& t, const zd* khat, const Cols& c,
                                int precond, int nb, const zd* v, long long vs, zd* X, zd* Y,
                                zd* S, zd* y, long long ys, const zd* V, long long ldj, int nv,
                                int nvmax, zd* partial, int nblk, zd* out, long long ostride,
                                const int* active, hipStream_t st);
hipError_t launch_operator_dots_f32(const Geo& g, const Trig& t, const zf* khat_f, const Cols& c,
                                    int precond, int nb, const zd* v, long long vs, zf* Xf,
                                    zf* Yf, zd* S, zd* y, long long ys, const zf* V,
                                    long long ldj, int nv, int nvmax, zd* partial, int nblk,
                                    zd* out, long long ostride, const int* active,
                                    hipStream_t st);
hipError_t launch_operator_dots_f32(const Geo& g, const Trig& t, const zf* khat_f, const Cols& c,
                                    int precond, int nb, const zf* v, long long vs, zf* Xf,
                                    zf* Yf, zd* S, zd* y, long long ys, const zf* V,
                                    long long ldj, int nv, int nvmax, zd* partial, int nblk,
                                    zd* out, long long ostride, const int* active,
                                    hipStream_t st);
hipError_t launch_operator_dots_f32(const Geo& g, const Trig& t, const zf* khat_f, const Cols& c,
                                    int precond, int nb, const zf* v, long long vs, zf* Xf,
                                    zf* Yf, zd* S, zf* y, long long ys, const zf* V,
                                    long long ldj, int nv, int nvmax, zd* partial, int nblk,
                                    zd* out, long long ostride, const int* active,
                                    hipStream_t st);
// out[i] = (float) in[i]
hipError_t launch_to_f32(const zd* in, zf* out, long long n, hipStream_t st);
// One single-layer family on a coefficient grid (inspection path).
hipError_t launch_single_family(const Geo& g, const Trig& t, const zd* khat, int family,
                                const zd* in, zd* X, zd* Y, zd* out, hipStream_t st);

// Krylov building blocks: vector r of a set at base + r n; basis vector i of right-hand
// side r at V + i ldj + r n.
// The basis V is double, or single precision (zf) in the mixed-precision solve; w, h and
// the results stay double.
hipError_t launch_dots(const zd* V, long long ldj, int nv, int nvmax, const zd* w, long long n,
                       int nb, zd* partial, int nblk, zd* out, long long ostride, zd* acc,
                       long long astride, const int* active, hipStream_t st);
hipError_t launch_dots(const zf* V, long long ldj, int nv, int nvmax, const zd* w, long long n,
                       int nb, zd* partial, int nblk, zd* out, long long ostride, zd* acc,
                       long long astride, const int* active, hipStream_t st);
// First update fused with the second pass's dot products (nv <= 8): w -= V h, then
// out = V^H w (updated), also added into acc, as launch_dots writes them.
hipError_t launch_update_dots(const zd* V, long long ldj, int nv, int nvmax, const zd* h,
                              long long hstride, zd* w, long long n, int nb, zd* partial,
                              int nblk, zd* out, long long ostride, zd* acc, long long astride,
                              const int* active, hipStream_t st);
hipError_t launch_update_dots(const zf* V, long long ldj, int nv, int nvmax, const zd* h,
                              long long hstride, zd* w, long long n, int nb, zd* partial,
                              int nblk, zd* out, long long ostride, zd* acc, long long astride,
                              const int* active, hipStream_t st);
hipError_t launch_update(const zd* V, long long ldj, int nv, const zd* h, long long hstride,
                         zd* w, long long n, int nb, const int* active, hipStream_t st);
hipError_t launch_update(const zf* V, long long ldj, int nv, const zd* h, long long hstride,
                         zd* w, long long n, int nb, const int* active, hipStream_t st);
hipError_t launch_norm2(const zd* w, long long n, int nb, double* partial, int nblk, double* out,
                        const int* active, hipStream_t st);
hipError_t launch_scale_copy(const zd* w, const double* nrm2, zd* v, long long n,
                             long long vstride, int nb, const int* active, hipStream_t st);
hipError_t launch_sub(const zd* b, const zd* w, zd* r, long long total, hipStream_t st);
hipError_t launch_givens(const Krylov& kv, int j, int nb, hipStream_t st);
// w_r -= V h_r, with nblk partial sums of |w_r|^2 in npart[r * nblk + b].
hipError_t launch_update_norm(const zd* V, long long ldj, int nv, const zd* h, long long hstride,
                              zd* w, long long n, int nb, double* npart, int nblk,
                              const int* active, hipStream_t st);
hipError_t launch_update_norm(const zf* V, long long ldj, int nv, const zd* h, long long hstride,
                              zd* w, long long n, int nb, double* npart, int nblk,
                              const int* active, hipStream_t st);
// ... with w stored in single precision (updated in double precision).
hipError_t launch_update_norm(const zf* V, long long ldj, int nv, const zd* h, long long hstride,
                              zf* w, long long n, int nb, double* npart, int nblk,
                              const int* active, hipStream_t st);
// |w_r|^2 (from nparts partials, or kv.nrm2 when nparts == 0), Givens step of column j
// (j >= 0), v_r = w_r / |w_r| (v_r at v + r vstride) and z_r = P^{-1} v_r (z_r at z + r n),
// each of w, v, z stored in double or single precision as the overload says.
hipError_t launch_next_vector(const Geo& g, const Krylov& kv, int j, const double* npart,
                              int nparts, const zd* w, zd* v, long long vstride, const Cols& c,
                              zd* z, int nb, hipStream_t st);
hipError_t launch_next_vector(const Geo& g, const Krylov& kv, int j, const double* npart,
                              int nparts, const zd* w, zf* v, long long vstride, const Cols& c,
                              zd* z, int nb, hipStream_t st);
hipError_t launch_next_vector(const Geo& g, const Krylov& kv, int j, const double* npart,
                              int nparts, const zd* w, zf* v, long long vstride, const Cols& c,
                              zf* z, int nb, hipStream_t st);
hipError_t launch_next_vector(const Geo& g, const Krylov& kv, int j, const double* npart,
                              int nparts, const zf* w, zf* v, long long vstride, const Cols& c,
                              zf* z, int nb, hipStream_t st);
hipError_t launch_solve_y(const Krylov& kv, int nb, hipStream_t st);
// Restart bookkeeping on the device.  init: |b_r| = sqrt(nrm2[r]), iterations zero.
// cycle_start (after nrm2[r] = |r_r|^2 of the current residual): relative residual, stop
// test (tol, max_iter), active/incycle flags, g = (|r_r|, 0, ...), cycle threshold
// thr = max(tol |b_r|, inner |r_r|).  cycle_end: iterations += columns built.
hipError_t launch_krylov_init(const Krylov& kv, int nb, hipStream_t st);
hipError_t launch_cycle_start(const Krylov& kv, int nb, int max_iter, double inner,
                              hipStream_t st);
hipError_t launch_cycle_end(const Krylov& kv, int nb, hipStream_t st);
hipError_t launch_combine(const Geo& g, const Krylov& kv, const zd* V, long long ldj,
                          const Cols& c, zd* x, int nb, hipStream_t st);
hipError_t launch_combine(const Geo& g, const Krylov& kv, const zf* V, long long ldj,
                          const Cols& c, zd* x, int nb, hipStream_t st);

// Back-substitution and synthesis of levels [j0, j1) of nr fields: solution r at
// xap + r xs, field r at eout + r es; tbuf holds 3 nr (j1 - j0) staging levels.
hipError_t launch_synthesis(const Geo& g, const Trig& t, const zd* pi_d, const zd* theta_d,
                            const zd* pi_n, const zd* xap, long long xs, int nr, int j0, int j1,
                            zd* tbuf, zd* eout, long long es, hipStream_t st);
// Aperture transforms E^1(u), E^2(u) for nq queries: per-block partial sums (2 complex per
// block and query); solution r at xall + r * n.
hipError_t launch_rcs_partial(const Geo& g, const zd* xall, long long n, const RcsQuery* queries,
                              int nq, zd* partial, int nblk, hipStream_t st);
hipError_t launch_pack(const Geo& g, const zd* xpad, zd* xcompact, hipStream_t st);
hipError_t launch_unpack(const Geo& g, const zd* xcompact, zd* xpad, hipStream_t st);

// Direct solve for small cavities (n = 3 NM, column-major n x n matrices).
hipError_t launch_unit_vectors(long long n, long long k0, int nb, zd* x, hipStream_t st);
hipError_t launch_dense_fix(const Geo& g, zd* A, hipStream_t st);
// Gauss-Jordan inversion with partial pivoting of A (overwritten; B is scratch of the same
// size): *result = (P A)^{-1} (A or B), piv[k] = row exchanged with row k at step k, or -1
// from the first step that found no nonzero pivot on.
hipError_t launch_gj_invert(zd* A, zd* B, long long n, int* piv, zd** result, hipStream_t st);
// x_r = F (P b_r) for r < nb, perm[i] = source row of (P b)_i; pb: nb x n scratch.
hipError_t launch_dense_apply(const zd* F, const int* perm, long long n, const zd* b, int nb,
                              zd* pb, zd* x, hipStream_t st);
hipError_t launch_add(zd* x, const zd* y, long long total, hipStream_t st);

}  // namespace cav
