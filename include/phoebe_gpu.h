/*
 * phoebe_gpu.h -- C ABI of the MI355X (gfx950) electron-phonon interpolation
 * and scattering-rate library.
 *
 * The operations follow the Phoebe paper (arXiv:2111.14999):
 *   - electron bands by Wannier interpolation: H^W(k) = sum_R e^{ik.R} H(R)
 *     and its diagonalisation U_k^dagger H^W(k) U_k = diag(eps_k)
 *     (Electron Properties);
 *   - phonons: D(q) = sum_R V2(0|R) e^{iq.R}, D z = (hbar omega)^2 z
 *     (Phonon Properties, dynamical matrix and its eigenvalue equation);
 *   - the Wannier-to-Bloch interpolation of the el-ph coupling with the
 *     (1/2 m omega)^{1/2} factor (Electron Properties, definition of g and its
 *     interpolation from g(Re, Rp)), computed as the two phase sums of the
 *     Kokkos (Interaction) section;
 *   - the electron lifetime 1/tau_kb (Transport Methods, electron BTE) with
 *     Gaussian smearing (Dirac delta and Smearing) and an energy window
 *     (Band structure classes).
 *
 * Conventions (every entry point):
 *   - simple-cubic lattice, a = 1 A: k, q and R in crystal coordinates;
 *     phases are e^{+i 2 pi k.R};
 *   - units: energies eV, masses amu, force constants eV/A^2, g(Re,Rp) eV/A,
 *     hbar omega = 0.0646541513 sqrt(lambda) eV, phonon length
 *     l_{s,q nu} = sqrt(4.18015928e-3 / (2 M_s hbar omega)) A, Gamma in eV;
 *   - arrays are C order; complex numbers are interleaved (re, im) doubles;
 *   - "device" pointers are HIP device memory of the handle's device, "host"
 *     pointers are ordinary host memory read before the call returns;
 *   - the caller owns every input and output buffer; the handle owns its
 *     workspace (device memory grown on demand up to the budget given at
 *     creation);
 *   - every call validates its arguments before launching anything and
 *     returns a status; after an error no output is defined and
 *     phoebe_gpu_last_error() describes it;
 *   - work is enqueued on the given HIP stream (hipStream_t passed as void*,
 *     NULL = default stream).  Calls return after enqueueing except where a
 *     host-visible result (a count) is documented as synchronising;
 *   - a handle is used by one host thread at a time.
 */
#ifndef PHOEBE_GPU_H
#define PHOEBE_GPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PHOEBE_GPU_ABI_VERSION 2

typedef struct {
    double re, im;
} phoebe_c128;

typedef enum {
    PHOEBE_OK = 0,
    PHOEBE_E_INVALID = -1,     /* bad argument: null pointer, size, enum, mesh */
    PHOEBE_E_NOMEM = -2,       /* workspace budget or device allocation exhausted */
    PHOEBE_E_DEVICE = -3,      /* a HIP runtime call failed */
    PHOEBE_E_UNSUPPORTED = -4, /* valid request outside what the kernels implement */
    PHOEBE_E_NUMERIC = -5      /* non-finite value met where a finite one is required */
} phoebe_status;

/* Arithmetic of the phase and rotation contractions.  Band structure,
 * occupations, smearing and the rate accumulation are FP64 in every mode. */
typedef enum {
    PHOEBE_FP64 = 0,   /* FP64 MFMA, FP64 accumulation */
    PHOEBE_FP32 = 1,   /* operands rounded to FP32, FP32 MFMA, FP32 accumulation */
    PHOEBE_BF16X3 = 2, /* FP32 operands split hi+lo in BF16, 3 products, FP32 accumulation */
    PHOEBE_BF16X6 = 3, /* FP32 operands split in 3 BF16 pieces, 6 products, FP32 accumulation */
    PHOEBE_BF16 = 4    /* MLP only: FP32 storage, BF16 operands, FP32 accumulation */
} phoebe_precision;

/* Long-range (polar) part of the coupling of a polar crystal (Electron
 * Properties: the split g = g^S + g^L and the long-range expression):
 *   g^L_{nu n m}(k, q) = i L(q, nu) [U_k^dagger U_{k+q}]_{n m},
 *   L(q, nu) = 4 pi (e^2/(4 pi eps0)) sum_s l_{s,q nu}
 *              sum_{G: q+G != 0} [(q+G) . Z*_s . z^s_{q nu}] e^{-(q+G).eps.(q+G)/(4 alpha)}
 *                                / [(q+G) . eps_inf . (q+G)],
 * with (q+G) the Cartesian vector 2 pi (q + G) (1/A), G over the integer box
 * [-g_max, g_max]^3, e^2/(4 pi eps0) = 14.399645 eV A and V = 1 A^3. */
typedef struct {
    const double *born;         /* host [nat, 3, 3] Born effective charges Z*_{s, a b}, units of e */
    double eps_inf[9];          /* high-frequency dielectric tensor, row major (positive definite) */
    double alpha;               /* Gaussian damping of the G sum, A^-2 (> 0) */
    int32_t g_max;              /* half-width of the G box (0 <= g_max <= 8) */
} phoebe_polar;

/* One crystal.  Integer lattice-vector lists are HOST pointers; the tensors
 * are DEVICE pointers. */
typedef struct {
    int32_t n_wannier;          /* nW >= 1 */
    int32_t n_atoms;            /* nat >= 1; nModes = 3 nat, phonon index s*3+alpha */
    int32_t n_rh;               /* number of Hamiltonian lattice vectors */
    const int32_t *rh;          /* host   [n_rh, 3] */
    const phoebe_c128 *h_r;     /* device [n_rh, nW, nW]  <0 n|H|R m>, eV */
    int32_t n_rd;               /* number of force-constant lattice vectors */
    const int32_t *rd;          /* host   [n_rd, 3] */
    const double *phi_r;        /* device [n_rd, nModes, nModes]  V2(0 s a|R s' b), eV/A^2 */
    const double *mass;         /* device [nat] amu */
    int32_t n_re;               /* electron lattice vectors of g */
    const int32_t *re;          /* host   [n_re, 3] */
    int32_t n_rp;               /* phonon lattice vectors of g */
    const int32_t *rp;          /* host   [n_rp, 3] */
    const phoebe_c128 *g_rr;    /* device [n_re, n_rp, nModes, nW, nW] g(Re,Rp), eV/A;
                                   first Wannier index pairs with k, second with k+q */
    const phoebe_polar *polar;  /* host, nullable: a polar crystal's long-range coupling, added
                                   to g by interp_g, the rate and the linewidth sums */
} phoebe_system;

/* Smearing of the energy-conserving delta (Dirac delta and Smearing). */
typedef enum {
    PHOEBE_SMEAR_GAUSSIAN = 0, /* fixed width sigma */
    PHOEBE_SMEAR_ADAPTIVE = 1  /* adaptive Gaussian: a width per transition (k n) -> (k+q m),
                                  sigma_t = max(sigma, (A / sqrt 12) |(v_nk - v_m,k+q) . 2 pi / N|),
                                  the velocity difference (eV A) taken per axis times the
                                  mesh step 2 pi / N_beta (1/A) of that axis, A = adaptive_scale */
} phoebe_smearing;

/* Parameters of the rate sum.  States with win_lo < eps < win_hi are kept;
 * modes with hbar omega < omega_min are left out (and get l = 0). */
typedef struct {
    double mu;        /* chemical potential, eV */
    double kT;        /* k_B T, eV (> 0) */
    double sigma;     /* Gaussian smearing: delta(x) = exp(-x^2/sigma^2)/(sqrt(pi) sigma), > 0;
                         with PHOEBE_SMEAR_ADAPTIVE the floor of the per-transition width */
    double win_lo;    /* energy window, eV */
    double win_hi;
    double omega_min; /* eV, >= 0 */
    int32_t smearing;       /* phoebe_smearing */
    double adaptive_scale;  /* A of the adaptive width (> 0; 1 is the plain reading) */
} phoebe_rate_params;

/* ABI version of the loaded library (PHOEBE_GPU_ABI_VERSION it was built with). */
int32_t phoebe_gpu_abi_version(void);

/* Create a handle on HIP device `device`; the workspace may grow to
 * workspace_budget_bytes (0 = 90% of the device's free memory at creation).
 * Errors: PHOEBE_E_INVALID (null out-pointer, bad device), PHOEBE_E_DEVICE. */
phoebe_status phoebe_gpu_create(int device, size_t workspace_budget_bytes, void **handle);

/* Release the handle and its workspace (synchronises the device first).
 * NULL is accepted and ignored. */
phoebe_status phoebe_gpu_destroy(void *handle);

/* Text of the last error on this handle ("" if none); valid until the next
 * call on the handle.  handle may be NULL (then: last error of create). */
const char *phoebe_gpu_last_error(void *handle);

/* Electron bands at arbitrary wavevectors (Electron Properties: back Fourier
 * transform of H(R) and its diagonalisation).
 *   k_frac    device [nk, 3] crystal coordinates
 *   eps_out   device [nk, nW] ascending eigenvalues, eV
 *   u_out     device [nk, nW, nW] eigenvectors as columns (nullable)
 * Only sys->n_wannier, n_rh, rh, h_r are read.  nk = 0 is a no-op. */
phoebe_status phoebe_gpu_electron_bands(void *handle, const phoebe_system *sys,
                                        const double *k_frac, int64_t nk,
                                        double *eps_out, phoebe_c128 *u_out, void *stream);

/* Phonon modes at arbitrary wavevectors (Phonon Properties: dynamical matrix,
 * mass-weighted as D/sqrt(M_s M_s'), and its eigenvalue equation).
 *   q_frac    device [nq, 3]
 *   omega_out device [nq, nModes] hbar omega = 0.0646541513 sqrt(max(lambda, 0)), eV,
 *             in ascending lambda
 *   z_out     device [nq, nModes, nModes] orthonormal eigenvectors as columns (nullable)
 * Only n_atoms, n_rd, rd, phi_r, mass are read.  nq = 0 is a no-op. */
phoebe_status phoebe_gpu_phonon_modes(void *handle, const phoebe_system *sys,
                                      const double *q_frac, int64_t nq,
                                      double *omega_out, phoebe_c128 *z_out, void *stream);

/* Interpolated el-ph coupling for every pair of a k list and a q list
 * (Electron Properties, definition of g and its Wannier interpolation; the
 * two phase sums of the Kokkos section):
 *   g_{nu n m}(k, q) = sum_{s alpha} [U_k^dagger G_{s alpha}(k,q) U_{k+q}]_{n m}
 *                      z_{s alpha, nu}(q) l_{s, q nu},
 *   G(k, q) = sum_{Re, Rp} e^{i 2 pi (k.Re + q.Rp)} g(Re, Rp),
 * with l = 0 for hbar omega < omega_min.
 *   k_frac  device [nk, 3];  q_frac device [nq, 3]
 *   g_out   device [nk, nq, nModes, nW, nW]  index (i, j, nu, n at k, m at k+q)
 *   eps_k   device [nk, nW] (nullable); eps_kq device [nk, nq, nW] (nullable);
 *   omega_q device [nq, nModes] (nullable)
 * Eigenvector phases are those of the library's eigensolver, so g itself is
 * defined up to a phase per band and per mode (|g|^2 summed over degenerate
 * states is gauge-free).  nk = 0 or nq = 0 is a no-op.
 * Errors: PHOEBE_E_INVALID, PHOEBE_E_NOMEM, PHOEBE_E_UNSUPPORTED (nW > 32 or
 * nModes > 32), PHOEBE_E_DEVICE. */
phoebe_status phoebe_gpu_interp_g(void *handle, const phoebe_system *sys,
                                  const double *k_frac, int64_t nk,
                                  const double *q_frac, int64_t nq,
                                  double omega_min, phoebe_precision prec,
                                  phoebe_c128 *g_out, double *eps_k, double *eps_kq,
                                  double *omega_q, void *stream);

/* phoebe_gpu_interp_g with the q list the full mesh q_mesh (host [3]): the
 * nq = N0 N1 N2 points q = (i0/N0, i1/N1, i2/N2) in linear order
 * (i0 N1 + i1) N2 + i2; g_out, eps_kq and omega_q are indexed by that order.
 * On the mesh the phase e^{i 2 pi q.Rp} is a product of three per-axis factors
 * (the Electron Properties interpolation of g, applied one lattice axis at a
 * time as for phoebe_gpu_scatter_rates' factorised sums), so in FP64 and FP32,
 * where the Rp box [-rmax, rmax]^3 is at most 31 wide and at most half as wide
 * as the Rp count, the sum over Rp is taken axis by axis; the result is the same
 * sum up to the order of the additions.  Otherwise (split-BF16, other Rp lists)
 * it is the dense contraction of phoebe_gpu_interp_g.  When every k is a point
 * of the mesh (k N_d integral to 1e-9), every k + q is one too: the bands at
 * the pairs are then the mesh's, one eigensolve per mesh point gathered per pair
 * (equal to the per-pair eigensolves up to rounding and the eigenvector phases).
 * k_frac is read back to the host once.
 * Errors as phoebe_gpu_interp_g; PHOEBE_E_INVALID for q_mesh NULL or below 1. */
phoebe_status phoebe_gpu_interp_g_mesh(void *handle, const phoebe_system *sys,
                                       const double *k_frac, int64_t nk,
                                       const int32_t q_mesh[3], double omega_min,
                                       phoebe_precision prec, phoebe_c128 *g_out,
                                       double *eps_k, double *eps_kq, double *omega_q,
                                       void *stream);

/* Scattering rates Gamma_nk = hbar/tau_nk on a uniform mesh (Transport
 * Methods, electron lifetime; Gaussian smearing; energy window):
 *   Gamma_nk = 2 pi sum_q w_q sum_m sum_nu |g_{nu n m}(k,q)|^2
 *       [(n_{q nu}+1-f_{m,k+q}) delta(eps_nk-eps_{m,k+q}-hbar omega_{q nu})
 *      + (n_{q nu}+f_{m,k+q})   delta(eps_nk-eps_{m,k+q}+hbar omega_{q nu})],
 * f Fermi-Dirac(mu, kT), n Bose-Einstein(kT), k+q folded onto the mesh.
 * With sys->polar set, g includes the long-range part g^L (see phoebe_polar);
 * with par->smearing = PHOEBE_SMEAR_ADAPTIVE each delta takes its own width
 * (see phoebe_smearing; 1/sigma_t inside the sum).
 *   k_mesh    host [3], the k mesh; point (i0,i1,i2) has linear index
 *             (i0 N1 + i1) N2 + i2 (third coordinate fastest)
 *   q_mesh    host [3], the q mesh.  k + q must be a point of the k mesh, so
 *             the two must be equal: a q mesh different from the k mesh
 *             returns PHOEBE_E_UNSUPPORTED
 *   k_idx     device [nk] mesh linear indices of the k points to evaluate, or
 *             NULL: every mesh k with a state in the window, ascending
 *   q_off, q_idx, q_w: NULL for the full q mesh with w_q = 1/N_q; otherwise
 *             explicit weighted q lists per evaluated k in CSR form:
 *             q_off device int64 [nk+1], q_idx device int32 [q_off[nk]],
 *             q_w device double [q_off[nk]] (only with k_idx != NULL)
 *   gamma_out device [rows, nW]; row a belongs to the a-th evaluated k; bands
 *             outside the window get 0.  rows = nk, or N_k (= N0 N1 N2)
 *             capacity when k_idx is NULL
 *   band_mask device uint8 [rows, nW], 1 = in window (nullable)
 *   kept_k_out device int32 [rows] mesh index of each row (nullable)
 *   n_kept_out host int64 (nullable): number of rows written.  When k_idx is
 *             NULL the call synchronises the stream once, after the window
 *             step, to learn this count.
 * Workspace: in the factorised full-mesh form the first Re-axis intermediate is
 * kept for every k0 plane of the call when the handle's budget allows it
 * (n0 planes of (2 r_e + 1)^2 n_rp nModes nW^2 elements; 39 GB for a 40^3 mesh,
 * nW = 16, 15 modes, 343 Re and Rp in FP64), so g(Re,Rp) is read once per call;
 * under a smaller budget it is kept per batch and g is read once per batch.  The
 * states are then taken in sub-batches whose Rp-axis intermediates stay under
 * 16 GB or a quarter of the budget, whichever is less.  The results are the
 * same bit for bit.
 * Errors: PHOEBE_E_INVALID (mesh < 1, sigma <= 0, kT <= 0, enum, pointers),
 * PHOEBE_E_NOMEM, PHOEBE_E_UNSUPPORTED (nW > 32, nModes > 32, q_mesh != k_mesh,
 * polar or adaptive smearing with another precision than FP64, split-BF16 with
 * nModes*nW > 512),
 * PHOEBE_E_NUMERIC (finiteness checks on, see phoebe_gpu_set_check_finite),
 * PHOEBE_E_DEVICE. */
phoebe_status phoebe_gpu_scatter_rates(void *handle, const phoebe_system *sys,
                                       const int32_t k_mesh[3], const int32_t q_mesh[3],
                                       const int32_t *k_idx, int64_t nk,
                                       const int64_t *q_off, const int32_t *q_idx,
                                       const double *q_w,
                                       const phoebe_rate_params *par, phoebe_precision prec,
                                       double *gamma_out, uint8_t *band_mask,
                                       int32_t *kept_k_out, int64_t *n_kept_out,
                                       void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): phoebe_gpu_scatter_rates
 * with the same arguments, results and errors, whose workspace is a static
 * device array of phoebe_gpu_noalloc_scratch_bytes() bytes (256 MiB less one
 * flag block) instead of the handle's workspace.  The call performs no device
 * allocation or free (and takes no timing records).  A problem whose workspace
 * does not fit fails with PHOEBE_E_NOMEM before any launch; the planner sizes
 * its batches to the scratch, so moderate meshes fit (the tables of a 40^3
 * mesh with nW = 16 alone do not).  Every call on one device shares that
 * device's array and leaves its contents behind: calls that overlap on one
 * device (two streams, two threads, two handles) race and must be ordered by
 * the caller.  The array's address is resolved once per device when the first
 * handle on that device is created. */
phoebe_status phoebe_gpu_scatter_rates_noalloc(void *handle, const phoebe_system *sys,
                                               const int32_t k_mesh[3], const int32_t q_mesh[3],
                                               const int32_t *k_idx, int64_t nk,
                                               const int64_t *q_off, const int32_t *q_idx,
                                               const double *q_w,
                                               const phoebe_rate_params *par,
                                               phoebe_precision prec, double *gamma_out,
                                               uint8_t *band_mask, int32_t *kept_k_out,
                                               int64_t *n_kept_out, void *stream);

/* Table cache of the rate path (off by default).  With it on, the electron
 * bands and eigenvectors and the phonon frequencies, eigenvectors and Bose
 * occupations that a rate call (phoebe_gpu_scatter_rates, _rate_terms,
 * _delta_weights, _phonon_linewidth) builds on its mesh are kept in a device
 * buffer of the handle (N (16 nW^2 + 8 nW + 16 nModes^2 + 16 nModes) bytes),
 * and a later call reuses them instead of rebuilding them when the system's
 * h_r, phi_r and mass pointers, its lattice lists, nW, n_atoms, the mesh,
 * omega_min and kT are all the same (results are bitwise the same as without
 * the cache).  The match is on pointers: a caller that rewrites those arrays
 * in place must turn the cache off (which frees it) or back on (which empties
 * it) before the next call.  Not used by phoebe_gpu_scatter_rates_noalloc. */
phoebe_status phoebe_gpu_set_table_cache(void *handle, int enable);

/* Testing aid for callers' error handling: with at > 0, the at-th HIP runtime
 * call the library checks from now on (on this handle) is reported as failed
 * although it succeeded; the call in progress then waits for the device and
 * returns PHOEBE_E_DEVICE with a last-error message ending in "(injected)".  The
 * injection fires once; the handle stays usable.  at = 0 disarms it, at < 0 is
 * PHOEBE_E_INVALID. */
phoebe_status phoebe_gpu_set_fault_injection(void *handle, int64_t at);

/* Usable bytes of the static scratch of phoebe_gpu_scatter_rates_noalloc. */
size_t phoebe_gpu_noalloc_scratch_bytes(void);

/* Batched form: many independent systems (different nW, nModes, lattice-vector
 * sets and meshes) evaluated together (Transport Methods, electron lifetime,
 * per system exactly as phoebe_gpu_scatter_rates over the full q mesh with
 * k_idx = NULL).  A plan builds every system's band and phonon tables, windows
 * and kept-state lists, picks each system's tile shape with an autotuner (the
 * candidates are timed on the device; choices are read from and written to
 * tune_cache, a small JSON file, when it is not NULL), and captures one
 * hipGraph: stage 1 and the U_k fold of every system, then persistent
 * kernels (one per tile shape in use) that drain work queues of (system,
 * state, q tile) tasks, then the per-system reductions.  Only PHOEBE_FP32
 * contractions (complex64) are offered; tables, eigensolves, occupations and
 * rate sums are FP64.  Unless the handle's mesh-sum mode is
 * PHOEBE_MESH_SUM_DIRECT, every system that phoebe_gpu_scatter_rates would sum
 * in the factorised form (the automatic rule of phoebe_gpu_set_mesh_sum on its
 * full q mesh) is taken out of the graph and run by phoebe_gpu_batched_run as
 * one plain rate call (FP32, the handle's workspace, the band and phonon tables
 * the plan built) after the graph; such systems report tq = tn = 0 in
 * phoebe_gpu_batched_info.
 *   systems   host [n_sys] (their tensors are device pointers, used until the
 *             plan is destroyed)
 *   meshes    host [n_sys, 3];  params host [n_sys]
 *   n_kept_out host [n_sys] (nullable): kept k per system
 * The plan call synchronises the stream.  Errors as phoebe_gpu_scatter_rates,
 * PHOEBE_E_UNSUPPORTED for other precisions. */
phoebe_status phoebe_gpu_batched_plan(void *handle, const phoebe_system *systems, int32_t n_sys,
                                      const int32_t *meshes, const phoebe_rate_params *params,
                                      phoebe_precision prec, const char *tune_cache,
                                      void **plan, int64_t *n_kept_out, void *stream);

/* Launch the plan's graph on `stream`, then copy each system's rates to
 * gamma_out[i] (device [n_kept_i, nW_i], rows in ascending mesh order of the
 * kept k; bands outside the window get 0).  gamma_out is a host array of
 * n_sys device pointers; it or any entry may be NULL (no copy). */
phoebe_status phoebe_gpu_batched_run(void *plan, double *const *gamma_out, void *stream);

/* Plan facts: tile shape of system `sys` (q rows = 16 tq, column tiles per
 * wave tn), its kept states, the total number of queue tasks, and the time
 * the autotuner spent. Any out-pointer may be NULL. */
phoebe_status phoebe_gpu_batched_info(void *plan, int32_t sys, int32_t *tq, int32_t *tn,
                                      int64_t *n_states, int64_t *n_tasks, double *tune_ms);

/* Release a plan (synchronises the device). NULL is accepted. */
phoebe_status phoebe_gpu_batched_destroy(void *plan);

/* Per-term output of the rate sum (FP64): for each kept state of the given k
 * points, terms[state, q, nu] = 2 pi/(sqrt(pi) sigma) x sum_m |g_{nu n m}(k,q)|^2
 *   [(n+1-f) e^{-(x-w)^2/sigma^2} + (n+f) e^{-(x+w)^2/sigma^2}]
 * over the full q mesh, so that Gamma_nk = (1/N_q) sum_{q,nu} terms.  These are
 * the integrand samples the learned proposal is trained on.  dweights
 * (nullable, same shape) receives the same expression with |g|^2 = 1 (the
 * smearing weight D), so terms / D is the |g|^2 the proposal network fits.
 *   k_idx    device [nk] (required);  gamma_out device [nk, nW] as scatter_rates
 *   terms    device [max_states, N_q, nModes]; dweights the same
 *   st_row, st_band device int32 [max_states] (nullable): row (index into
 *            k_idx) and band of each state, states ordered by row then band
 *   max_states capacity of the per-state outputs (nk*nW always suffices); if the
 *            window holds more states the call fails with PHOEBE_E_INVALID
 *            before writing any of them
 *   n_states host (nullable): number of states written
 * Synchronises the stream.  Terms of final bands outside the window-wide
 * non-zero range (see phoebe_gpu_scatter_rates) are exactly zero. */
phoebe_status phoebe_gpu_rate_terms(void *handle, const phoebe_system *sys, const int32_t mesh[3],
                                    const int32_t *k_idx, int64_t nk,
                                    const phoebe_rate_params *par, double *gamma_out,
                                    double *terms, double *dweights, int32_t *st_row,
                                    int32_t *st_band, int64_t max_states, int64_t *n_states,
                                    void *stream);

/* Smearing weights D[state, q, nu] alone (see phoebe_gpu_rate_terms): band and
 * phonon tables, window and states as in the rate path, no coupling work;
 * dweights, st_row, st_band and max_states as there.  gamma_scratch device
 * [nk, nW] is zeroed.  Synchronises the stream. */
phoebe_status phoebe_gpu_delta_weights(void *handle, const phoebe_system *sys,
                                       const int32_t mesh[3], const int32_t *k_idx, int64_t nk,
                                       const phoebe_rate_params *par, double *dweights,
                                       int32_t *st_row, int32_t *st_band, int64_t max_states,
                                       int64_t *n_states, double *gamma_scratch, void *stream);

/* Learned q-proposal network: a multilayer perceptron with n_in inputs, `depth`
 * hidden layers of `width` silu units and one linear output.  Parameters are
 * packed layer by layer as W_l [out, in] (row major) then b_l [out].
 * PHOEBE_BF16: float storage, BF16 operands on MFMA, FP32 accumulation;
 * PHOEBE_FP64: double storage and arithmetic (for checking gradients).
 * Returns the number of parameters (-1 for a bad shape). */
int64_t phoebe_gpu_mlp_param_count(int32_t n_in, int32_t width, int32_t depth);

/* out[b] = network(X[b]);  X device [batch, n_in], out device [batch]. */
phoebe_status phoebe_gpu_mlp_forward(void *handle, phoebe_precision prec, const void *params,
                                     int32_t n_in, int32_t width, int32_t depth, const void *X,
                                     int64_t batch, void *out, void *stream);

/* Mean squared error L = (1/B) sum_b (network(X_b) - target_b)^2 and its
 * gradient with respect to the packed parameters (backpropagation).
 *   grad device [param_count] (same storage type as params); loss host (nullable,
 *   synchronises the stream when set). */
phoebe_status phoebe_gpu_mlp_grad(void *handle, phoebe_precision prec, const void *params,
                                  int32_t n_in, int32_t width, int32_t depth, const void *X,
                                  const void *target, int64_t batch, void *grad, double *loss,
                                  void *stream);

/* One Adam step (Kingma & Ba, bias-corrected; step >= 1) on FP32 parameters
 * with FP32 first and second moments m, v (device [n]). */
phoebe_status phoebe_gpu_mlp_adam(void *handle, float *params, const float *grad, float *m,
                                  float *v, int64_t n, int32_t step, double lr, double beta1,
                                  double beta2, double eps, void *stream);

/* Network inputs of samples given by mesh indices k_idx, q_idx, band energy
 * eps and mode nu (device arrays [batch]), e = (eps - e0)/escale:
 *   n_harm = 0: x = [k (3 crystal coords), e, q (3), one-hot(nu)]  (7 + n_modes)
 *   n_harm > 0: x = [e, one-hot(nu), and for h = 1..n_harm: cos and sin of
 *               2 pi h k_d (d = 0..2), then of 2 pi h q_d]       (1 + n_modes + 12 n_harm)
 * X device [batch, phoebe_gpu_mlp_feature_count(n_modes, n_harm)] (float for
 * BF16, double for FP64).  n_harm in [0, 16]. */
int32_t phoebe_gpu_mlp_feature_count(int32_t n_modes, int32_t n_harm);
phoebe_status phoebe_gpu_mlp_features(void *handle, phoebe_precision prec, const int32_t mesh[3],
                                      int32_t n_modes, int32_t n_harm, const int32_t *k_idx,
                                      const double *eps, const int32_t *q_idx, const int32_t *nu,
                                      int64_t batch, double e0, double escale, void *X,
                                      void *stream);

/* Importance-sampling lists from the learned proposal.  For each k (host
 * k_idx[i], host band energy eps_k[i] of its targeted state, smearing weights
 * dweights + i N_q nModes of that state) the proposal is
 *   p_raw(q) = sum_nu D[q, nu] e^{net(k, eps, q, nu)}
 * where the network (BF16, inputs as phoebe_gpu_mlp_features with n_harm)
 * estimates ln(|g|^2 + c) and is evaluated only where
 * D > d_threshold x max D; with params = NULL the network factor is 1 (the
 * smearing-only proposal, the method without the network).  The proposal is
 * p = (1 - mix) p_raw / sum p_raw + mix / N_q; mix in (0, 1] keeps every q
 * possible, which keeps the estimate unbiased.  S points are drawn by inverse
 * CDF of the given uniforms (device [nk, S] in [0, 1)) and weighted
 * w = 1 / (N_q S p(q)): q_off device int64 [nk+1], q_idx device int32 [nk S],
 * q_w device [nk S], ready for phoebe_gpu_scatter_rates.  Every k is handled
 * in the same pass (one selection over all rows, the network over the listed
 * entries of every k in batches, one sampler work-group per k); nk N_q nModes
 * must stay below 2^31 (else PHOEBE_E_INVALID: split the k list).
 * Synchronises once. */
phoebe_status phoebe_gpu_propose_q(void *handle, const int32_t mesh[3], int32_t n_modes,
                                   int32_t n_harm, const int32_t *k_idx, const double *eps_k, int64_t nk,
                                   const double *dweights, const float *params, int32_t width,
                                   int32_t depth, double e0, double escale, double d_threshold,
                                   double mix, int32_t S, const double *uniforms, int64_t *q_off,
                                   int32_t *q_idx, double *q_w, void *stream);

/* Phonon scattering rate from the electron-phonon interaction, the el-ph
 * term on the diagonal of the phonon scattering matrix (Transport Methods,
 * phonon BTE), with the paper's replacement f_kb - f_{k+q,b'} ~ (df/de) hbar omega:
 *   P_{q nu} = (2 pi / N_k) n (n + 1) hbar omega_{q nu}
 *              sum_{k, b, b'} |g_{nu b b'}(k, q)|^2 f_kb (1 - f_kb) / kT
 *              delta(eps_kb - eps_{b',k+q} - hbar omega_{q nu}),
 * n = n(omega_{q nu}); b runs over the states of the window at every k of the
 * k mesh, b' over all bands; modes with hbar omega < omega_min get P = 0.  g,
 * the smearing (fixed or adaptive) and the window are those of
 * phoebe_gpu_scatter_rates, and so is the evaluation: the coupling of each
 * kept state is formed once and its terms go to the linewidth of every q.
 *   k_mesh, q_mesh host [3] (equal; otherwise PHOEBE_E_UNSUPPORTED)
 *   p_out     device [N_q, nModes] eV
 *   gamma_out device [N_k, nW] (nullable): the electron rates of the same pass,
 *             rows as scatter_rates with k_idx = NULL
 *   n_kept_out host (nullable): kept k points summed over
 * The sum over states is taken in a fixed order: two calls give equal bits.
 * Synchronises the stream once (to learn the kept count).  FP64 only.
 * Errors as phoebe_gpu_scatter_rates; PHOEBE_E_UNSUPPORTED for other
 * precisions. */
phoebe_status phoebe_gpu_phonon_linewidth(void *handle, const phoebe_system *sys,
                                          const int32_t k_mesh[3], const int32_t q_mesh[3],
                                          const phoebe_rate_params *par, phoebe_precision prec,
                                          double *p_out, double *gamma_out, int64_t *n_kept_out,
                                          void *stream);

/* Electron group velocities (Electron Properties, Velocity): the velocity
 * operator v_a = U_k^dagger (dH^W/dk_a) U_k with the analytic derivative
 * dH^W/dk_a = sum_R i R_a e^{i 2 pi k.R} H(R) (eV A, Cartesian R, a = 1 A);
 * a non-degenerate band's velocity is its diagonal element, a degenerate group
 * (|delta eps| < 1e-6 eV) has its block of each v_a diagonalised and its bands
 * take the eigenvalues in ascending order.
 *   k_frac device [nk, 3];  eps_out device [nk, nW] (nullable)
 *   v_out  device [nk, nW, 3] eV A
 * Only n_wannier, n_rh, rh, h_r are read.  nk = 0 is a no-op. */
phoebe_status phoebe_gpu_velocities(void *handle, const phoebe_system *sys, const double *k_frac,
                                    int64_t nk, double *eps_out, double *v_out, void *stream);

/* The q-dependent factor L(q, nu) of the long-range coupling (see
 * phoebe_polar), with l = 0 for hbar omega < omega_min.
 *   q_frac device [nq, 3];  l_out device [nq, nModes] complex, eV
 * Needs sys->polar and the force constants.  nq = 0 is a no-op. */
phoebe_status phoebe_gpu_polar_factor(void *handle, const phoebe_system *sys, const double *q_frac,
                                      int64_t nq, double omega_min, phoebe_c128 *l_out,
                                      void *stream);

/* Anharmonic force constants of a crystal for the 3-phonon coupling: the
 * harmonic part as in phoebe_system and the third derivatives
 * Phi3(s a R, s' b R', s'' c 0) with the third displacement in the reference
 * cell.  Lattice lists are HOST pointers, tensors DEVICE pointers. */
typedef struct {
    int32_t n_atoms;
    int32_t n_rd;  const int32_t *rd;  const double *phi_r;  const double *mass;
    int32_t n_r1;  const int32_t *r1;  /* host [n_r1, 3]: R of the first displacement */
    int32_t n_r2;  const int32_t *r2;  /* host [n_r2, 3]: R' of the second displacement */
    const double *phi3;                /* device [n_r1, n_r2, nModes, nModes, nModes] eV/A^3 */
} phoebe_system3;

/* Interpolated 3-phonon coupling for every pair of a q list and a q' list
 * (Phonon Properties, the Fourier transform of the third derivative; the
 * generic contraction of the Kokkos section, the sum over R taken at fixed q,
 * then the sum over R' at each q'):
 *   V3(q nu, q' nu', q'' nu'') = sum_{R, R'} sum_{sa, s'b, s''c} Phi3(s a R, s' b R', s'' c 0)
 *       e^{-i 2 pi (q.R + q'.R')} z*_{sa,nu}(q) l z*_{s'b,nu'}(q') l' z*_{s''c,nu''}(q'') l'',
 * q'' = -q - q', l the phonon length of each mode (0 below omega_min).
 *   q_frac device [nq, 3];  qp_frac device [nqp, 3]
 *   v3_out device [nq, nqp, nModes, nModes, nModes] complex, eV (nu, nu', nu'')
 *   omega_q [nq, nModes], omega_qp [nqp, nModes], omega_qpp [nq, nqp, nModes]
 *           device (nullable)
 * Eigenvector phases are the library's, so V3 is defined up to a phase per
 * mode; |V3|^2 summed over degenerate modes is phase-free.
 * Errors: PHOEBE_E_INVALID, PHOEBE_E_NOMEM, PHOEBE_E_UNSUPPORTED (nModes > 30),
 * PHOEBE_E_DEVICE. */
phoebe_status phoebe_gpu_interp_v3(void *handle, const phoebe_system3 *sys, const double *q_frac,
                                   int64_t nq, const double *qp_frac, int64_t nqp,
                                   double omega_min, phoebe_c128 *v3_out, double *omega_q,
                                   double *omega_qp, double *omega_qpp, void *stream);

/* Counter-based random numbers: Philox-4x64 with 10 rounds (Salmon, Moraes,
 * Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).
 * Element i of the stream (seed, offset) is the first 64-bit word w0 of the
 * block Philox(counter = (offset + i, 0, 0, 0), key = (seed, 0)), so a stream is
 * the same on any device and launch shape, and disjoint offsets never overlap.
 *   uniform: out[i] = (w0 >> 11) 2^-53, a double in [0, 1)
 *   randint: out[i] = floor(uniform * hi), in [0, hi), 1 <= hi <= 2^31 - 1
 * out device [n].  n = 0 is a no-op. */
phoebe_status phoebe_gpu_philox_uniform(void *handle, uint64_t seed, uint64_t offset, int64_t n,
                                        double *out, void *stream);
phoebe_status phoebe_gpu_philox_randint(void *handle, uint64_t seed, uint64_t offset, int64_t n,
                                        int64_t hi, int32_t *out, void *stream);

/* Parameters of a new network (layout as phoebe_gpu_mlp_param_count): each
 * weight of layer l uniform in (-1/sqrt(in_l), 1/sqrt(in_l)) from the Philox
 * stream (seed, 0) in packing order, biases 0.  params device (float for
 * PHOEBE_BF16, double for PHOEBE_FP64). */
phoebe_status phoebe_gpu_mlp_init(void *handle, phoebe_precision prec, void *params, int32_t n_in,
                                  int32_t width, int32_t depth, uint64_t seed, void *stream);

/* Training set of the learned proposal from the method's own terms (see
 * phoebe_gpu_rate_terms): the entries (state, q, nu) with
 * D > d_threshold x max_{q,nu} D of their state are selected; each is kept
 * with probability min(1, max_samples / n_selected), decided by the Philox
 * uniform (seed, flat index); a kept entry gets the target
 *   y = ln(T / D + c),  c = c_frac x mean over the selected entries of T / D.
 *   terms, dweights device [n_states, N_q, nModes]
 *   st_row, st_band device [n_states]: row and band of each state
 *   out_state, out_q, out_nu device int32 [cap]; out_y device float [cap]
 *   n_out host: entries written (at most cap; entries beyond cap are dropped,
 *         in flat-index order); c_out host (nullable): the c used
 * Synchronises the stream. */
phoebe_status phoebe_gpu_training_set(void *handle, const double *terms, const double *dweights,
                                      int64_t n_states, int64_t n_q, int32_t n_modes,
                                      double d_threshold, double c_frac, int64_t max_samples,
                                      uint64_t seed, int32_t *out_state, int32_t *out_q,
                                      int32_t *out_nu, float *out_y, int64_t cap, int64_t *n_out,
                                      double *c_out, void *stream);

/* Row gather: dst[i] = src[idx[i]] for rows of row_bytes bytes (a multiple
 * of 4); idx device int32 [n], each in [0, n_src).  For minibatches. */
phoebe_status phoebe_gpu_gather_rows(void *handle, const void *src, int64_t n_src,
                                     int64_t row_bytes, const int32_t *idx, int64_t n, void *dst,
                                     void *stream);

/* Optional input validation: when enabled, the calls that read a system
 * (electron_bands, phonon_modes, velocities, interp_g, scatter_rates,
 * phonon_linewidth, rate_terms) first scan h_r, phi_r, mass and g_rr for
 * NaN or infinity and return PHOEBE_E_NUMERIC, before any other launch, if
 * one holds one.  The scan reads every input once and synchronises. */
phoebe_status phoebe_gpu_set_check_finite(void *handle, int enable);

/* How phoebe_gpu_scatter_rates (and rate_terms) evaluate the sum over Rp on a
 * full q mesh in FP64.  DIRECT: one MFMA contraction over the Rp list per q
 * tile, as for q lists.  FACTORED: the phase e^{i2pi q.Rp} is a product of
 * three per-axis factors on a full mesh, so the sum is taken one axis at a
 * time over the box [-rmax, rmax]^3 holding the Rp list (zero where the list
 * has no vector); the result is the same sum up to the order of additions.
 * Needs FP64 or FP32, the full q mesh, |Rp components| <= 15, nW <= 32,
 * nModes <= 32, N0 <= 1024 and N1*N2 <= 65535.
 * AUTO (the default) takes FACTORED where it applies and the box width is at
 * most half the number of Rp vectors (the sum over Re is then factorised the
 * same way over its box).  Lists of q, the split-BF16 precisions and the
 * batched form always use DIRECT.  Returns PHOEBE_E_INVALID for an
 * unknown mode; scatter_rates returns PHOEBE_E_UNSUPPORTED when FACTORED is
 * forced where it does not apply. */
typedef enum {
    PHOEBE_MESH_SUM_AUTO = 0,
    PHOEBE_MESH_SUM_DIRECT = 1,
    PHOEBE_MESH_SUM_FACTORED = 2
} phoebe_mesh_sum;
phoebe_status phoebe_gpu_set_mesh_sum(void *handle, int32_t mode);

/* Kernel timing for measurement: when enabled, the named hot kernels are
 * bracketed by HIP events on the stream they run on; phoebe_gpu_kernel_time
 * returns the number of timed launches and their summed duration since the
 * last reset.  Names: "stage2_rates" (direct sum), "stage1_phase" (direct sum over
 * Re), "stage1_axes" (factorised sum over Re), "axis_transforms" and "line_rates"
 * (factorised sum over Rp), "bands_fft", "eig_jacobi".  Timing synchronises the stream at the end of each call. */
phoebe_status phoebe_gpu_set_timing(void *handle, int enable);
phoebe_status phoebe_gpu_kernel_time(void *handle, const char *name,
                                     int64_t *launches, double *total_ms);
phoebe_status phoebe_gpu_reset_timing(void *handle);
/* Algorithmic HBM bytes the library recorded for the timed launches of a
 * kernel since the last reset (0 where it records none; "stage1_axes" records
 * the g(Re,Rp) read, its two intermediates written and read once, and G). */
phoebe_status phoebe_gpu_kernel_bytes(void *handle, const char *name, double *bytes);

#ifdef __cplusplus
}
#endif

#endif /* PHOEBE_GPU_H */
