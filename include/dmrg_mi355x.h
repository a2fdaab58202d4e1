/*
 * dmrg_mi355x: two-site DMRG effective-Hamiltonian path for MI355X (gfx950).
 *
 * The DMRG node of the paper maps active-space integrals (h_act, B^Q_act) to a
 * converged matrix-product state (Sec. II.C); its sweep is a two-site solve of
 * the effective Hamiltonian with a matrix-free Davidson against an MPO, followed
 * by SVD decimation to the bond dimension and a discarded weight
 * tau = sum of squared discarded singular values (Sec. II.H, Fig. 2).  The
 * two-electron integrals enter through Cholesky vectors,
 * (pq|rs) = sum_Q B^Q_pq B^Q_rs (Sec. II.A).  The active space is
 * (N_el, n_act) in the sector with fixed particle number and S_z (Sec. II.F).
 *
 * Conventions for every call:
 *  - Host pointers are borrowed for the duration of the call and copied.
 *  - Device pointers must be on the solver's device; work is ordered on the
 *    stream given at solver creation (a hipStream_t, may be NULL = default).
 *    Calls that return host values synchronise that stream.
 *  - Matrices are row-major, double precision.
 *  - Every function returns a dmrg_status; on failure dmrg_last_error() gives
 *    a message (thread-local, valid until the next call on the thread).  No
 *    C++ exception crosses this boundary.
 *  - One solver per thread; a solver must not be used concurrently.
 *
 * Storage of block-sparse tensors (quantum numbers (N, 2 S_z)):
 *  - A bond is a list of sectors (N, 2Sz, dim) sorted ascending by (N, 2Sz).
 *  - Site states s = 0..3 are |0>, |alpha>, |beta>, |alpha beta> with quantum
 *    numbers (0,0), (1,+1), (1,-1), (2,0); spin orbitals are ordered
 *    0a,0b,1a,1b,... (the Jordan-Wigner order of the MPS).
 *  - A three-leg tensor (site tensor: 4 physical states; two-site vector at
 *    sites (k, k+1): 16 states s = 4 s1 + s2) is stored slab by slab: for each
 *    left sector in bond order, a row-major m_left x W matrix whose column
 *    ranges are the blocks of the physical states in order whose right sector
 *    (left QN + state QN) exists, each m_right wide.
 */
#ifndef DMRG_MI355X_H
#define DMRG_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dmrg_problem dmrg_problem; /* opaque */
typedef struct dmrg_solver dmrg_solver;   /* opaque */
typedef struct dmrg_mlp dmrg_mlp;         /* opaque: preconditioner network */

typedef enum {
  DMRG_OK = 0,
  DMRG_EINVAL = -1,   /* invalid argument (non-symmetric h or B, bad sizes, ...) */
  DMRG_ENOMEM = -2,   /* device allocation failed */
  DMRG_EHIP = -3,     /* HIP / ROCm library failure */
  DMRG_ENOCONV = -4,  /* Davidson did not reach the tolerance (outputs still filled) */
  DMRG_ESECTOR = -5,  /* empty or inconsistent quantum-number sector */
  DMRG_ESTATE = -6    /* call out of order (e.g. no MPS / step not prepared) */
} dmrg_status;

typedef enum { DMRG_FP64 = 0, DMRG_FP32 = 1, DMRG_BF16 = 2 } dmrg_precision;
/* The two-site Davidson's run-time-selectable preconditioner family (Sec. III):
 * DIAG (Jacobi: (theta - D)^-1 r, with the deflation penalty's diagonal when
 * lower states are held), LEARNED (the network's correction, judged against the
 * exact residual with DIAG as fallback), OLSEN (the diagonal correction less its
 * component along (D - theta)^-1 x) and SHIFT_INVERT (up to 5 steps of projected
 * conjugate gradients on (1 - xx^T)(H - theta)(1 - xx^T) t = -r, preconditioned by
 * the projected diagonal, ended by a non-positive curvature, at pcg_rtol |r| or
 * after pcg_steps steps (dmrg_options, default 0.1 and 5); each step costs one
 * sigma product, counted in the matvecs). */
typedef enum {
  DMRG_PRECOND_DIAG = 0,
  DMRG_PRECOND_LEARNED = 1,
  DMRG_PRECOND_OLSEN = 2,
  DMRG_PRECOND_SHIFT_INVERT = 3
} dmrg_precond;

typedef struct {
  int M;               /* bond dimension (kept states per bond) */
  int n_states;        /* roots, state-averaged when > 1 (1..8) */
  const double* weights; /* n_states state-averaging weights (>= 0, normalised to sum 1), NULL = equal */
  double davidson_tol; /* ||H_eff x - theta x||_2 per root, with ||x|| = 1 */
  int max_iter;        /* Davidson iterations per step */
  int max_subspace;    /* Davidson subspace size (<= 64) */
  int precision;       /* dmrg_precision of the sigma products in Davidson */
  int precond;         /* dmrg_precond */
  unsigned long long seed; /* initial MPS and extra-root start vectors */
  double tie_rtol;     /* truncation never splits singular values closer than tie_rtol * s_1 */
  double cut_rtol;     /* when truncating, singular values <= cut_rtol * s_1 go first; nothing is
                          dropped while all states fit in M */
  int verbose;         /* 0 quiet, 1 per step, 2 per Davidson iteration (stderr) */
  long long sigma_chunk_bytes; /* bound on the sigma intermediates T (bytes; 0 = none): left factors
                                  are taken in chunks whose T fits, phase A and B run per chunk and
                                  phase B adds into sigma; less memory, more launches (slower) */
  int pcg_steps;       /* DMRG_PRECOND_SHIFT_INVERT: most inner CG steps per correction (>= 1) */
  double pcg_rtol;     /* ... and it stops once the inner residual is <= pcg_rtol * |r| (>= 0) */
  double trunc_tol;    /* > 0: per-bond adaptive bond dimension (Sec. II.H, dynamically adapted
                          per-bond M): each truncation keeps the fewest states whose discarded
                          weight is <= trunc_tol of the total (a cluster at that cut kept whole
                          while M allows), at least m_min and at most M; 0: fixed M */
  int m_min;           /* lower bound of the adaptive bond dimension (>= 1) */
} dmrg_options;

/* Fills *o with defaults: M=256, 1 state, tol 1e-10, 200 iterations, subspace
 * 32, FP64, diagonal preconditioner, seed 1, tie_rtol 1e-10, cut_rtol 1e-14,
 * unbounded sigma intermediates, 5 inner PCG steps to 0.1 |r|, fixed M
 * (trunc_tol 0, m_min 1). */
void dmrg_options_default(dmrg_options* o);

/* Active-space problem (Sec. II.A): n_orb spatial orbitals, n_alpha / n_beta
 * electrons (S_z = (n_alpha - n_beta)/2), h[n_orb*n_orb] one-electron integrals,
 * B[n_chol*n_orb*n_orb] Cholesky vectors B^Q_pq (row-major over Q, p, q),
 * e_core a constant added to energies.  h and every B^Q must be symmetric to
 * 1e-12 (else DMRG_EINVAL).  Builds the Cholesky-channel MPO on the host. */
dmrg_status dmrg_problem_create(int n_orb, int n_alpha, int n_beta, int n_chol, const double* h,
                                const double* B, double e_core, dmrg_problem** out);
void dmrg_problem_destroy(dmrg_problem* p);

/* MPO inspection (host only, no GPU needed).  dims[0..n_orb] receives the MPO
 * bond dimension of every cut.  dmrg_mpo_site_nnz gives the number of entries
 * W_k[a][b] = c * O (O a 4x4 site operator); dmrg_mpo_site copies them out:
 * a[i], b[i] channel indices at cuts k and k+1, c[i] coefficient, op[16*i..]
 * the row-major 4x4 operator <s|O|s'>.  Caller-owned arrays of nnz entries. */
dmrg_status dmrg_mpo_dims(const dmrg_problem* p, int* dims);
dmrg_status dmrg_mpo_site_nnz(const dmrg_problem* p, int site, int* nnz);
dmrg_status dmrg_mpo_site(const dmrg_problem* p, int site, int* a, int* b, double* c, double* op);

/* Solver on the current device with a seeded right-canonical random MPS (made
 * on the host: creation allocates no device memory; the MPS reaches the device
 * on the first call that needs device state).  Without a workspace the solver
 * allocates its device buffers (environments, MPS, plans, Davidson basis) with
 * hipMalloc as it needs them; after dmrg_workspace_attach every solver buffer,
 * rocBLAS's workspace included, is carved from the attached memory. */
dmrg_status dmrg_solver_create(const dmrg_problem* p, const dmrg_options* o, void* hip_stream,
                               dmrg_solver** out);
void dmrg_solver_destroy(dmrg_solver* s);

/* Device workspace (the paper's engine runs on one preallocated slab carved by
 * the library, Sec. III).  dmrg_workspace_query writes the bytes to attach for
 * the work ahead: an estimate from the current bonds and MPO (environments of
 * every cut, the largest step's sigma intermediates and Davidson basis, the MPS
 * and plans) before any workspace is attached; with one attached, at least 1.25
 * times its peak use, and after a call failed with DMRG_ENOMEM at least 1.25
 * times (what was in use + the request that did not fit).
 * dmrg_workspace_attach hands the library dev_ptr[0..bytes) (device memory on
 * the solver's device, caller-owned, e.g. a torch tensor; >= 1 MiB): the
 * solver's state (MPS, bonds, centre tensors, settings, statistics) moves into
 * it and every later solver buffer comes from it; the previous workspace (or
 * the library's own buffers) is released, so the caller may free the old slab
 * when the call returns.  Cached plans and environments are rebuilt on demand.
 * When a later call needs more than is free it fails with DMRG_ENOMEM (nothing
 * allocated): query again, attach a larger slab and repeat the call.  The
 * memory must stay valid until the solver is destroyed or another workspace is
 * attached.  The preconditioner network (dmrg_mlp) and the stand-alone calls
 * (dmrg_block_gemm, dmrg_measure_peaks) allocate their own memory. */
dmrg_status dmrg_workspace_query(const dmrg_solver* s, size_t* bytes);
dmrg_status dmrg_workspace_attach(dmrg_solver* s, void* dev_ptr, size_t bytes);

/* Replace the MPS.  n_sec[c] (c = 0..n_orb) sectors per bond, concatenated
 * sector tables sec[3*i] = N, sec[3*i+1] = 2Sz, sec[3*i+2] = dim; data = all
 * site tensors concatenated in the slab layout (host, double).  Bond 0 must be
 * the single vacuum sector, bond n_orb the single target sector. */
dmrg_status dmrg_set_mps(dmrg_solver* s, const int* n_sec, const int* sec, const double* data);

/* Current bond tables: n_sec[0..n_orb] and up to cap sector triples. */
dmrg_status dmrg_get_bonds(const dmrg_solver* s, int* n_sec, int* sec, int cap);

/* The current MPS, the forward result of the DMRG node (Sec. II.C: integrals
 * to the converged MPS), in the layout dmrg_set_mps takes: n_sec[0..n_orb]
 * (always written), the concatenated sector triples into sec (when not NULL;
 * sec_cap sectors must hold them all, else DMRG_EINVAL), and every site tensor
 * concatenated in slab layout into data (host, when not NULL; data_cap
 * doubles must hold them all, else DMRG_EINVAL).  *data_size receives the
 * number of doubles; call with sec = data = NULL to size the buffers.  After
 * a step or sweep the centre tensor of root 0 sits on the site the last step
 * moved to; the other sites are orthonormal. */
dmrg_status dmrg_export_mps(dmrg_solver* s, int* n_sec, int* sec, int sec_cap, double* data, int64_t data_cap,
                            int64_t* data_size);

/* Environments and plan for the two-site step on sites (k, k+1) of the current
 * MPS (any gauge): the left block, the two sites and the right block of the
 * decimation step (Fig. 2, Sec. II.H), contracted against the MPO.  *n
 * receives the two-site vector length.  Builds missing environments (their
 * update is the MPO contraction of Sec. II.H) and the sigma plan; host
 * planning plus GPU work, synchronises the stream. */
dmrg_status dmrg_prepare(dmrg_solver* s, int k, int64_t* n);

/* sigma = H_eff psi for step k: the matrix-free two-site effective Hamiltonian
 * against the MPO (Sec. II.H, Fig. 2), never formed densely; the two-electron
 * part enters through the Cholesky vectors (Sec. II.A).  The effective
 * Hamiltonian excludes e_core.  psi, sigma: device arrays of n doubles, the
 * two-site slab layout of step k (n must equal the length dmrg_prepare
 * returns, else DMRG_EINVAL; step k is prepared first when it is not).
 * precision: DMRG_FP64 (fp64 MFMA), DMRG_FP32 (fp32 MFMA) or DMRG_BF16 (bf16
 * inputs, fp32 accumulation); the output is always fp64.  If flops is not NULL
 * it receives the floating-point operations the launches execute (unpadded
 * block products).  Stream-ordered; the call waits for the kernels to time
 * them. */
dmrg_status dmrg_sigma(dmrg_solver* s, int k, int precision, int64_t n, const double* psi, double* sigma,
                       double* flops);

/* Diagonal of H_eff of step k (the Jacobi / diagonal member of the two-site
 * Davidson's preconditioner family, Sec. III) into a device array of n doubles
 * (n as for dmrg_sigma).  Synchronises the device. */
dmrg_status dmrg_diag(dmrg_solver* s, int k, int64_t n, double* diag);

/* Two-site sweeps (Sec. II.H, Fig. 2: at every bond a matrix-free Davidson
 * solve of H_eff, then SVD decimation to M keeping chi_k states and discarding
 * tau): left-to-right then right-to-left, (n_orb-1) steps each.
 * energies[n_states] (host): final Davidson Ritz values + e_core; tau: the
 * largest discarded weight of the last sweep.  DMRG_ENOCONV if a step did not
 * reach the tolerance (results still written). */
dmrg_status dmrg_sweep(dmrg_solver* s, int n_sweeps, double* energies, double* tau);

/* One-site sweeps at the current bond dimensions (Sec. II.E: a truncated
 * two-site fixed point is not stationary on the tangent space of its own bond
 * dimension, so its Hellmann-Feynman gradient differs from the derivative of
 * its energy by an amount that tracks the discarded weight).  Every step
 * optimises one site inside the two-site space (Davidson on P H_eff P, P the
 * projector on that site's tensors with the neighbour fixed) and moves the
 * centre by SVD without truncation.  *energy (host): the last step's energy +
 * e_core; *tangent_residual (may be NULL): the largest first-iteration
 * residual of the last sweep, the norm of the largest block of the gauge-free
 * tangent gradient B_k = V_L X_k; once it is ~0, dmrg_grad is the exact
 * gradient of the variational energy at this bond dimension.  One state; the
 * MPS must be right-orthonormal from site 1 (as after dmrg_sweep or a previous
 * call; DMRG_ESTATE if the centre is elsewhere).  DMRG_ENOCONV as dmrg_sweep. */
dmrg_status dmrg_stationarize(dmrg_solver* s, int n_sweeps, double* energy, double* tangent_residual);

/* One two-site step on sites (k, k+1) (the decimation step of Fig. 2): Davidson
 * on H_eff, SVD truncation to M, environment update; direction 0 moves the
 * center right (k -> k+1), 1 moves it left.  A sweep is steps 0..n_orb-2 in
 * direction 0 then n_orb-2..0 in 1.
 * The orthogonality centre must be on site k or k+1 (after solver creation it
 * is site 0; each step leaves it on the site it moved to; after dmrg_set_mps
 * the gauge is the caller's): else DMRG_ESTATE.
 * energies[n_states]: Ritz values + e_core; tau: discarded weight. */
dmrg_status dmrg_step(dmrg_solver* s, int k, int direction, double* energies, double* tau);

/* The SVD decimation of step k (Fig. 2: keep chi_k, discard tau = the sum of
 * the squared discarded singular values) applied to caller-given two-site
 * vectors instead of Davidson's: psi is a device array of n_states * n doubles
 * (root r at r * n; n as for dmrg_sigma).  psi is read as a matrix with rows
 * (left sector, s1) and columns (s2, right sector), block diagonal in the
 * middle-bond sector; singular values of all sectors (of the weighted
 * concatenation of the roots when n_states > 1) are sorted together and the
 * largest M kept, never splitting values closer than tie_rtol * s_1 and, when
 * truncating, dropping those <= cut_rtol * s_1 first (nothing is dropped while
 * all fit).  Updates bond k+1, sites k and k+1 and the centre like dmrg_step
 * (same centre requirement).  Outputs (host): *tau, *n_kept, and the kept
 * singular values in descending order into sv[0..min(sv_cap, n_kept)) when sv
 * is not NULL.  The singular values are square roots of eigenvalues of the
 * sector density matrices: their squares are exact to rounding (~1e-16 of the
 * norm), small values relatively less. */
dmrg_status dmrg_truncate(dmrg_solver* s, int k, int direction, int64_t n, const double* psi, double* tau,
                          double* sv, int sv_cap, int* n_kept);

/* <Psi|H|Psi>/<Psi|Psi> + e_core of the current MPS: per root when the centre
 * tensors of a sweep are present (centre on site 0), else energies[0] for the
 * MPS as stored (any gauge). */
dmrg_status dmrg_energy(dmrg_solver* s, double* energies);

/* Excited states by penalty deflation (Sec. II.F: lower converged MPS kept
 * resident and projected into every two-site optimisation through overlap
 * environments).  dmrg_deflate_add copies a lower state Phi (same active space
 * and sector; bonds and site tensors in the layout dmrg_set_mps takes, host
 * memory) to the device; from then on every Davidson solve of the solver uses
 * H_eff + sum_j weight_j |phi_j><phi_j| / <Phi_j|Phi_j>, phi_j the projection of
 * Phi_j into the step's two-site space, and the diagonal preconditioner adds
 * the penalty's diagonal.  Energies returned by dmrg_step / dmrg_sweep are those
 * of H (the Ritz value minus the penalty's expectation).  weight (Ha) must be
 * finite, positive and larger than the gap from the lower state to the target,
 * else the target may keep a component of the lower state (dmrg_overlap shows
 * it).  At most 32 lower states; DMRG_EINVAL on a malformed MPS or a zero norm.
 * dmrg_sigma and dmrg_diag stay those of H_eff alone.  The dual penalty of
 * Eq. (dualpen) is zero on every state of the (N, S_z) sector the solver works
 * in, so it needs no term here.  dmrg_deflate_clear drops all lower states. */
dmrg_status dmrg_deflate_add(dmrg_solver* s, const int* n_sec, const int* sec, const double* data, double weight);
dmrg_status dmrg_deflate_clear(dmrg_solver* s);

/* Projection of lower state j (added order) into the two-site space of step k,
 * unscaled (Phi as given): phi[a s1 s2 b] = sum OL[a a'] Phi_k[a' s1 m]
 * Phi_{k+1}[m s2 b'] OR[b b'] with the fp64 overlap environments OL (sites < k)
 * and OR (sites > k+1) of the current MPS.  phi: device array of n doubles
 * (n as for dmrg_sigma).  Synchronises the device. */
dmrg_status dmrg_deflate_project(dmrg_solver* s, int k, int j, int64_t n, double* phi);

/* <Psi|Phi_j> / (||Psi|| ||Phi_j||) of the current MPS and lower state j, a
 * transition overlap contracted over the whole chain in fp64 (host *overlap). */
dmrg_status dmrg_overlap(dmrg_solver* s, int j, double* overlap);

/* <S^2> of the current MPS (the spin guard of Sec. II.F: the solver fixes N
 * and S_z but is not spin-adapted, so S_z = 0 triplets share the sector):
 * <S_- S_+> + S_z (S_z + 1) through the solver's environment and sigma kernels
 * with a bond-dimension-4 MPO of S_- S_+.  s2[n_states] (host): per root when
 * the centre tensors of a sweep are present (centre on site 0), else s2[0] for
 * the MPS as stored (any gauge) and s2[1..] untouched. */
dmrg_status dmrg_s_squared(dmrg_solver* s, double* s2);

/* ---- Determinant space: CI vectors and (transition) RDMs ----------------
 * The device CI pipeline of Sec. III (colexicographic string ranks, string
 * enumeration, RDMs formed on the device) applied to MPS states: the RDMs of
 * the DMRG node's output (Sec. II.C: the node maps the integrals to the MPS and
 * its RDMs) and the transition RDMs between deflated roots (Sec. II.F).
 * Conventions: E_pq = sum_sigma a+_{p sigma} a_{q sigma}; a determinant is
 * (prod_{p in I_a} a+_{p alpha})(prod_{p in I_b} a+_{p beta})|0> with creators in
 * ascending orbital order, all alpha first; strings are ranked
 * colexicographically (rank = sum_t C(o_t, t+1) over sorted occupied orbitals);
 * a CI vector is the row-major matrix c[I_a][I_b], I_a < C(n, n_alpha),
 * I_b < C(n, n_beta).  Device memory is the caller's unless said otherwise; every call that takes
 * device CI vectors takes their length n, which must be C(n_orb,n_alpha) C(n_orb,n_beta)
 * (DMRG_EINVAL otherwise). */
/* String counts C(n_orb, n_alpha) and C(n_orb, n_beta).  Host only. */
dmrg_status dmrg_ci_dims(const dmrg_problem* p, int64_t* n_alpha_strings, int64_t* n_beta_strings);
/* The CI vector of an MPS, as stored (no normalisation): state 0 = the
 * solver's MPS (root 0), state j >= 1 = held state j-1 (dmrg_deflate_add).
 * c: device array of n = C(n,n_alpha) C(n,n_beta) doubles (DMRG_EINVAL
 * otherwise); at most 24 orbitals and n < 2^31.  Prefix and suffix partial
 * products meet at the middle bond as block GEMMs; temporaries are the
 * library's (workspace when one is attached). */
dmrg_status dmrg_mps_to_ci(dmrg_solver* s, int state, double* c, int64_t n);
/* Transition 1-/2-RDMs of device CI vectors bra, ket (may be the same pointer),
 * unnormalised:
 *   gamma[p*n+q] = <bra|E_pq|ket>,
 *   Gamma[((p*n+q)*n+r)*n+s] = <bra|E_pq E_rs|ket> - d_qr gamma_ps
 *     = sum_{sigma tau} <bra|a+_{p sigma} a+_{r tau} a_{s tau} a_{q sigma}|ket>,
 * overlap = <bra|ket>; host outputs (n^2, n^4 doubles, 1; each may be NULL).
 * At most 16 orbitals.  E_rs c for all rs in passes of determinants (a gather
 * kernel over string-excitation tables), then one fp64 MFMA product of
 * (n^2 + 1) x (n^2 + 1) over the determinants; runs on `stream` and returns
 * when the outputs are written. */
dmrg_status dmrg_ci_rdm12(const dmrg_problem* p, int64_t n, const double* bra, const double* ket, double* gamma, double* Gamma,
                          double* overlap, void* stream);
/* The all-active two-electron operator on a device CI vector (the fused
 * four-particle contraction of Sec. III: the two-electron block is contracted
 * into the ket, so <EEEE>-type densities contracted with it are three-body
 * densities of (bra, V ket) and the n^8 object is never formed):
 *   out = V c,  V = 1/2 sum_pqrs (pq|rs) E_pq E_rs,  (pq|rs) = sum_Q B^Q_pq B^Q_rs,
 * streamed through the problem's Cholesky factors (E_rs c for all rs, two
 * GEMMs over the factors, one gather sum); out: device, same length as c, not
 * aliasing it.  At most 16 orbitals. */
dmrg_status dmrg_ci_apply_v(const dmrg_problem* p, int64_t n, const double* c, double* out, void* stream);
/* Transition three-body density of device CI vectors (unnormalised):
 *   Gamma3[((((p*n+q)*n+r)*n+s)*n+t)*n+u] = <bra|E_pq E_rs E_tu|ket>
 * (host, n^6 doubles).  E_tu ket is kept for all tu, E_rs of each is formed in
 * passes of determinants and the fp64 MFMA split-K product with the bra's
 * copies accumulates the density.  At most 12 orbitals.  With ket = V c
 * (dmrg_ci_apply_v) it gives sum_vwxy (vw|xy)/2 <bra|E_pq E_rs E_tu E_vw E_xy|c>. */
dmrg_status dmrg_ci_rdm3(const dmrg_problem* p, int64_t n, const double* bra, const double* ket, double* Gamma3,
                         void* stream);
/* The same for MPS states (numbering as dmrg_mps_to_ci), each normalised:
 * gamma, Gamma and overlap of <bra|.|ket> / (|bra| |ket|). */
dmrg_status dmrg_rdm12(dmrg_solver* s, int bra_state, int ket_state, double* gamma, double* Gamma, double* overlap);

/* ---- Orbital entanglement and ordering (Sec. II.H: the pairwise mutual
 * information orders the lattice through the Fiedler vector) ---------------
 * From a device CI vector c (2..16 orbitals, any norm).  Two-orbital density
 * matrices: for each pair i < j (pairs in the order (0,1), (0,2), ..., (1,2),
 * ...), with the pair's spin orbitals moved to the front of every determinant
 * in the order (i alpha, j alpha, i beta, j beta), rho = Tr_rest |c><c| /
 * <c|c> over the 16 local states L = s_i + 4 s_j, s = n_alpha + 2 n_beta;
 * rho: host [n(n-1)/2][16][16].  Computed by one kernel over determinants and
 * pairs (each environment of a pair taken once, <= 4 amplitudes, fixed-order
 * sums). */
dmrg_status dmrg_orbital_rdm2(const dmrg_problem* p, int64_t n, const double* c, double* rho, void* stream);
/* One-orbital entropies s1[n] (natural log, from the diagonal one-orbital
 * density matrices) and mutual information I[n*n] = (s_i + s_j - s_ij) / 2
 * (zero diagonal), host outputs. */
dmrg_status dmrg_mutual_information(const dmrg_problem* p, int64_t n, const double* c, double* s1, double* I,
                                    void* stream);
/* The same density matrices and mutual information straight from the solver's
 * MPS (root 0, as stored, any active-space size the solver holds): every
 * element is the derivative of <Psi|O|Psi> by one closing entry of an MPO whose
 * channels open |t><s| on orbital i, carry the Jordan-Wigner parity across the
 * orbitals between, and close with |t_j><s_j| on orbital j, evaluated by the
 * per-site contractions of dmrg_grad; the MPO's environments hold 16 channels
 * per orbital to the left of each cut.  rho: host [n(n-1)/2][16][16], s1 / I as
 * dmrg_mutual_information; each may be NULL (s1 and I together). */
dmrg_status dmrg_mps_orbital_rdm2(dmrg_solver* s, double* rho, double* s1, double* I);
/* Orbital order from a mutual-information matrix (host only, 2..64 orbitals):
 * the eigenvector of the second-smallest eigenvalue of diag(sum_j I_ij) - I,
 * sign fixed so that its largest-magnitude component (first such) is
 * positive; order[n] lists the orbitals by ascending component (stable);
 * fiedler[n] (may be NULL) receives the vector.  Reorder h and B^Q by it (new
 * orbital t = old order[t]) for the next calculation. */
dmrg_status dmrg_fiedler_order(int n, const double* I, int* order, double* fiedler);

/* Integral gradient of the current MPS energy (Sec. II.C: the DMRG node's
 * adjoint; the MPS is held fixed, i.e. the Hellmann-Feynman term, exact for a
 * converged full-bond state; at truncated bond it is the gradient of
 * <Psi|H|Psi>/<Psi|Psi> for the MPS as it stands, Sec. II.E).  Every entry of h
 * and B is an independent variable:
 *   dE/dh_pq = gamma_pq = sum_sigma <a+_{p sigma} a_{q sigma}>,
 *   dE/dB^Q_pq = sum_rs Gamma'_pqrs B^Q_rs,
 *   Gamma'_pqrs = sum_{sigma tau} <a+_{p sigma} a+_{r tau} a_{s tau} a_{q sigma}>
 * (a symmetric parameterisation adds the (p,q) and (q,p) entries).
 * state_weights[n_states] (host, may be NULL = root 0 only): the output is
 * sum_r w_r dE_r; roots r > 0 need the centre tensors left by dmrg_step /
 * dmrg_sweep (else DMRG_ESTATE when their weight is non-zero).  Outputs (host,
 * caller-owned): dE_dh[n_orb*n_orb], dE_dB[n_chol*n_orb*n_orb] (row-major like
 * the inputs; may be NULL when n_chol = 0), energies[n_states] (may be NULL):
 * <Psi_r|H|Psi_r>/<Psi_r|Psi_r> + e_core of every root (0 for roots without a
 * centre tensor).  Leaves the environments of root 0 in place. */
dmrg_status dmrg_grad(dmrg_solver* s, const double* state_weights, double* dE_dh, double* dE_dB,
                      double* energies);

/* ---- Learned Davidson preconditioner ------------------------------------
 * The paper's two-site Davidson takes a run-time-selectable preconditioner
 * (Sec. III); this library adds a learned member.  A per-amplitude network
 *   y = W3 relu(W2 relu(W1 x + b1) + b2) + b3   (x: n_in features, width hidden)
 * maps 8 features of each amplitude of a correction to the correction itself:
 *   f0 r_i sqrt(n)/|r|, f1 e_i/s_b, f2 clip(s_b/e_i, -10, 10), f3 t_i sqrt(n)/|t|,
 *   f4 mean_b(e/s_b), f5 min_b(e/s_b), f6 log(block size)/10, f7 k/L,
 * with e = diag(H_eff) - theta, t_i = r_i/(theta - d_i) the diagonal candidate
 * (|theta - d_i| floored at 1e-8), b the dense block of the amplitude and s_b
 * the mean of |e| over it.  Weights are fp32; the hidden layer runs in bf16 on
 * the matrix cores inside Davidson.  Each learned candidate is judged: if it
 * is not finite or keeps less than 1e-3 of its norm after orthogonalisation
 * to the subspace, the diagonal candidate replaces it, and when three learned
 * iterations cut the exact residual norm by less than 10% the rest of the
 * step uses the diagonal candidate.  Convergence is always on the exact
 * residual.  Parameters are one fp32 vector: W1[width][n_in], b1[width],
 * W2[width][width], b2[width], W3[width], b3[1]. */

/* Network with He-normal weights (seeded) and zero biases; work on hip_stream. */
dmrg_status dmrg_mlp_create(int n_in, int width, unsigned long long seed, void* hip_stream, dmrg_mlp** out);
void dmrg_mlp_destroy(dmrg_mlp* m);
dmrg_status dmrg_mlp_num_params(const dmrg_mlp* m, int64_t* n);
/* Host parameter vectors of exactly num_params floats; set also resets Adam. */
dmrg_status dmrg_mlp_set_params(dmrg_mlp* m, const float* host, int64_t n);
dmrg_status dmrg_mlp_get_params(const dmrg_mlp* m, float* host, int64_t n);
/* y[rows] = net(X[rows][n_in]) (device fp32 arrays); precision DMRG_FP32 or
 * DMRG_BF16 (hidden layer with bf16 inputs, fp32 accumulation).  Synchronous. */
dmrg_status dmrg_mlp_forward(dmrg_mlp* m, int precision, const float* X, int64_t rows, float* y);
/* Training loss on n_seg segments of seg_len rows (device X[n_seg*seg_len][n_in],
 * target[n_seg*seg_len]): loss = mean over segments of 1 - cos(y_seg, target_seg)
 * (scale-free: Davidson ignores the scale of a correction), fp32 forward and
 * backward; the gradient is kept for dmrg_mlp_adam_step and copied to grad
 * (host, num_params floats) when grad is not NULL. */
dmrg_status dmrg_mlp_loss_grad(dmrg_mlp* m, const float* X, const float* target, int n_seg, int seg_len,
                               double* loss, float* grad);
/* Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with the last gradient. */
dmrg_status dmrg_mlp_adam_step(dmrg_mlp* m, double lr);
/* Preconditioner of later Davidson solves (dmrg_precond): DMRG_PRECOND_LEARNED
 * takes a network of n_in = 8 (borrowed: it must outlive its use by the
 * solver); the others ignore net. */
dmrg_status dmrg_set_precond(dmrg_solver* s, int precond, dmrg_mlp* net);
/* Training triples from later Davidson solves (root 0): at every iteration the
 * features of `sample` amplitudes (a seeded draw per step), and once the step
 * has converged the target Delta = P_perp psi* on the same amplitudes (psi* the
 * converged vector oriented along the iterate psi_i, P_perp projecting out
 * psi_i).  Steps that do not converge, or whose vector is shorter than
 * `sample`, record nothing.  capacity 0 stops recording. */
dmrg_status dmrg_record_triples(dmrg_solver* s, int capacity, int sample);
/* Copies up to cap recorded triples into device arrays X[cap][sample][8] and
 * target[cap][sample] (fp32), writes the count and empties the store. */
dmrg_status dmrg_take_triples(dmrg_solver* s, float* X, float* target, int cap, int* count);
/* The 8 features (device X[n][8], fp32) of the two-site step k for device
 * vectors r (residual) and d (diagonal of H_eff) and eigenvalue estimate theta;
 * n must be the step's two-site length (DMRG_EINVAL otherwise). */
dmrg_status dmrg_precond_features(dmrg_solver* s, int k, int64_t n, const double* r, const double* d, double theta,
                                  float* X);
/* One correction vector of the preconditioner family (Sec. III) at two-site step
 * k, as a Davidson iteration forms it: device vectors of the step's length n
 * (checked: DMRG_EINVAL otherwise),
 * x the Ritz vector (unit norm), r = H_eff x - theta x its residual, d the
 * diagonal of H_eff (dmrg_diag); t (device, n, caller-owned) receives
 * DMRG_PRECOND_DIAG: (theta - d)^-1 r (each |theta - d_i| floored at 1e-8),
 * DMRG_PRECOND_OLSEN: that minus (x.q_r / x.q_x) q_x with q_x = (theta - d)^-1 x,
 * DMRG_PRECOND_SHIFT_INVERT: the inner PCG of the shift-and-invert mode on the
 * step's H_eff in fp64 (without deflation penalties; the solver's pcg_steps and
 * pcg_rtol); *products (may be NULL)
 * receives the sigma products it made.  DMRG_PRECOND_LEARNED is rejected. */
dmrg_status dmrg_correction(dmrg_solver* s, int k, int mode, int64_t n, const double* x, const double* r, const double* d,
                            double theta, double* t, int* products);

/* Diagnostic export of an environment of the current MPS: side 0 = left block
 * (sites < cut), 1 = right block (sites >= cut).  Copies min(cap, size) doubles
 * of the channel arrays (channels grouped by quantum-number shift, each a list
 * of dense row-major blocks) to host and writes the full size to *size. */
dmrg_status dmrg_get_env(dmrg_solver* s, int cut, int side, double* host, int64_t cap, int64_t* size);

/* The block-GEMM engine on one block, for tests: C (M x N, ldc) = coef * op(A) op(B)
 * on the given stream.  mode 0: A M x K, B K x N; 1: A M x K, B N x K (B^T);
 * 2: A K x M (A^T), B K x N; all row-major device arrays.  precision
 * DMRG_FP64: double A, B, C; DMRG_FP32: float A, B, C; DMRG_BF16: bf16 bit
 * patterns (uint16) A, B, float C (modes 0 and 1). */
dmrg_status dmrg_block_gemm(int precision, int mode, int M, int N, int K, const void* A, int lda,
                            const void* B, int ldb, void* C, int ldc, double coef, void* hip_stream);

/* Allocation-free dmrg_block_gemm, for callers that cannot allocate device
 * memory (work under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments and result as dmrg_block_gemm; the tile
 * and item descriptors live in a fixed device array inside the library
 * (256 KiB per device, held until the process ends) instead of memory allocated
 * per call, so the call makes no hipMalloc / hipFree and no host-to-device copy.
 * Limit: the M x N output must fit 4096 tiles of 64 x 64 (e.g. M, N <= 4096),
 * else DMRG_EINVAL.  Stream-ordered: it returns once the work is enqueued on
 * hip_stream (dmrg_block_gemm synchronises).  Every call on one device shares
 * that device's descriptor array: calls that overlap on one device (other
 * streams or threads) race; calls in order on one stream do not. */
dmrg_status dmrg_block_gemm_noalloc(int precision, int mode, int M, int N, int K, const void* A, int lda,
                                    const void* B, int ldb, void* C, int ldc, double coef, void* hip_stream);

/* Device ceilings for roofline reports, measured on the current device: the
 * fp64 MFMA rate of a register-only loop of v_mfma_f64_16x16x4 (four
 * independent accumulators per wave, 8 waves per SIMD) and the bandwidth of a
 * streaming copy of `bytes` from src to dst (read + write bytes per second).
 * src and dst are caller-owned device buffers on the current device, 16-byte
 * aligned, bytes a multiple of 16 and >= 4 MiB (dst's first 4 MiB also take
 * the MFMA loop's results; both buffers' contents are overwritten / read).
 * Best of three timed runs after a warm-up, on hip_stream; blocks the calling
 * thread.  Outputs: *fp64_tflops in TFLOP/s, *copy_gbs in GB/s (1e9 B/s). */
dmrg_status dmrg_measure_peaks(void* hip_stream, const void* src, void* dst, size_t bytes, double* fp64_tflops,
                               double* copy_gbs);

/* Precision of the sigma products in later Davidson solves (dmrg_precision; the
 * option of the same name at creation).  fp64 is kept for the basis, the
 * subspace eigenproblem, the residual, the truncation and the environments.
 * The low-precision forms run refinement cycles: the subspace restarts from
 * Ritz vectors with fp64 products, new directions get fp32 / bf16 products,
 * and when the residual estimate has dropped by 1e-4, stalled, or passed the
 * tolerance the Ritz vectors get fp64 products again (defect correction).
 * Convergence is declared only on such an exact fp64 residual; when a cycle
 * cuts the exact residual by less than a factor 0.3, the rest of the step uses
 * fp64 products. */
dmrg_status dmrg_set_precision(dmrg_solver* s, int precision);

/* Profiling aid: the fp64 sigma kernels exist as two identical instantiations
 * each (phase A: gemm_f64_w32<0, 1 | 3, ...>; phase B: gemm_wg<double, 2 | 4>);
 * tag 0 (default) launches the first of each pair, tag 1 the second, so a
 * profiler can separate e.g. timed from untimed launches.  No effect on
 * results. */
dmrg_status dmrg_set_kernel_tag(dmrg_solver* s, int tag);

/* Run statistics (host doubles): [0] matvecs, [1] Davidson iterations,
 * [2] sigma ms, [3] env-update ms, [4] SVD ms, [5] sigma flops, [6] tau,
 * [7] max bond dimension, [8] preconditioner fallbacks, [9] 1 while every
 * Davidson solve so far reached the tolerance (0 after the first that did not),
 * [10] sigma phase-A ms (T = X psi), [11] sigma phase-B ms (long-K products),
 * [12] phase-A flops, [13] phase-B flops, [14] environment-update flops,
 * [15] fp64 refinements, [16] phase-B GEMM kernel ms alone (fp64; without the
 * split-K reduction), [17] dmrg_grad wall ms, [18] dmrg_grad flops (without
 * the environment updates it triggers), [19] step-preparation wall ms
 * (environments, factors, plans), [20] plan resolution and upload wall ms,
 * [21] Davidson wall ms, [22] step plans reused (a step's plan depends only on
 * its outer bonds and is kept per step; it is rebuilt when they change),
 * [23] phase-A flops executed, [24] phase-B flops executed, [25] sigma
 * products in low precision (fp32 / bf16); [15] counts the precision form's
 * refinement cycles (fp64 products of the Ritz vectors), [26] peak bytes in
 * use in the attached workspace (0 without one), [27] device allocations the
 * library made with hipMalloc since the workspace was attached (process-wide
 * count; -1 without a workspace), [28] host wall ms spent building step plans
 * (part of [19]), [29] host wall ms spent building environment-update plans.
 * Times of [2]-[4], [10], [11], [16] are HIP-event times on the solver stream
 * and flops count unpadded block products.  The sigma flops [5], [12], [13]
 * are algorithmic: every block product of the middle-cut factorisation (all
 * columns of every T_X, every item).  The executed counts [23], [24] are
 * lower: phase A skips T_X columns no item reads, and phase B merges items
 * that share their T slice (sum_j c_j T Y_j^T = T (sum_j c_j Y_j)^T).
 * n: capacity of out (up to 30 values are written). */
dmrg_status dmrg_get_stats(const dmrg_solver* s, double* out, int n);

const char* dmrg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DMRG_MI355X_H */
