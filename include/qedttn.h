/*
 * qedttn: tree-tensor-network node update for (3+1)D compact lattice QED
 * (Magnifico, Felser, Silvi, Montangero, arXiv:2011.10658) on AMD MI355X.
 *
 * C ABI.  Conventions shared by every entry point:
 *   - Every function returns an int status: QED_OK (0) on success, a
 *     negative QED_ERR_* on error, QED_NOT_CONVERGED (+1) as a warning.
 *     qed_last_error(ctx) returns a context-owned message for the last
 *     failure on that context (valid until the next call on it).
 *   - A context is single-threaded; separate contexts are independent.
 *   - Host pointers are borrowed for the duration of the call; output
 *     arrays are caller-allocated with the sizes stated below.
 *   - Device pointers passed in are owned by the caller and borrowed.
 *     Library-internal device memory comes from the registered allocator
 *     (stream-ordered HIP allocations by default) and is released by
 *     qed_destroy / the matching *_destroy.
 *   - All GPU work is enqueued on the registered stream (the null stream
 *     by default).  Functions that return host scalars synchronise it.
 *   - Floating-point state is real FP64 unless stated; GEMM-heavy steps
 *     can run in FP32 or BF16 with FP32 accumulation (qed_set_precision).
 *
 * Layout contract of a three-leg U(1) block tensor (legs l, r, p):
 *   each leg is a list of sectors with strictly ascending charges q and
 *   sizes n > 0.  The allowed blocks are the (l, r, p) sector triples with
 *   q_l + q_r - q_p = flux (node tensors: flux 0), sorted by (q_l, q_r)
 *   ascending; block b is stored at flat[off[b] .. off[b+1]) with off the
 *   int64 prefix sums of n_l n_r n_p, and the entry (i_l, i_r, i_p) of a
 *   block at (i_l * n_r + i_r) * n_p + i_p.
 * Layout of a block-sparse leg operator with charge shift delta (maps
 *   sector q to sector q + delta of the same leg): for every input sector
 *   in ascending order whose shifted charge is a sector of the leg, one
 *   dense row-major (n_{q+delta} x n_q) block, blocks concatenated.
 */
#ifndef QEDTTN_H
#define QEDTTN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    QED_OK = 0,
    QED_NOT_CONVERGED = 1,
    QED_ERR_INVALID_ARG = -1,
    QED_ERR_BAD_STATE = -2,
    QED_ERR_OOM = -3,
    QED_ERR_HIP = -4,
    QED_ERR_NONFINITE = -6,
    QED_ERR_UNSUPPORTED = -7,
    QED_ERR_IO = -8
};

/* Boundary readings for open lattices.  The paper runs open boundaries,
 * including finite charge density (Results, "Finite Density"), without
 * fixing the outward half-links.  ZERO_FLUX freezes each outward rishon
 * at k = 1 (E = 0; only Q = 0 exists); FREE_FLUX keeps it a free 3-state
 * mode with electric energy (g_e^2/2) E^2 and no penalty partner.
 * PERIODIC (the zero-charge transition, Results) wraps every axis of
 * extent >= 2; an axis of extent 1 has no links and its half-links are
 * frozen as under ZERO_FLUX.  With extent 2 the two sites of an axis are
 * joined by two distinct links (direct and wrapped).  Only Q = 0 exists. */
enum { QED_BC_OPEN_ZERO_FLUX = 0, QED_BC_OPEN_FREE_FLUX = 1, QED_BC_PERIODIC = 2 };

/* Arithmetic of the block GEMMs (H_eff matvec).  Lanczos, QR, the
 * environment renormalisation and energies are always FP64. */
enum { QED_FP64 = 0, QED_FP32 = 1, QED_BF16 = 2 };

typedef struct qed_ctx qed_ctx;
typedef struct qed_heff qed_heff;
typedef struct qed_heff_batch qed_heff_batch;

/* Per-sweep record (Methods, "Numerical Convergence": energy, penalty and
 * link-constraint error tracked along the optimisation). */
typedef struct {
    double energy;     /* energy after the last node update of the sweep  */
    double dE;         /* energy change against the previous sweep        */
    double nu;         /* penalty coefficient used in this sweep          */
    double deltaL;     /* sum over links of |<L_{x,mu} - 2>|              */
    double Q;          /* <total charge>                                  */
    double seconds;    /* wall time of the sweep                          */
    double flops;      /* algorithmic H_eff matvec flops in the sweep     */
    long long matvecs; /* H_eff applications in the sweep                 */
} qed_sweep_report;

/* ---------------------------------------------------------------- */
/* context                                                           */
/* ---------------------------------------------------------------- */

/* Create a context bound to HIP device `hip_device`.  hip_device < 0
 * creates a host-only context (model, tree and block-table queries
 * only; any GPU call on it returns QED_ERR_BAD_STATE).  *out is owned by
 * the caller and freed with qed_destroy. */
int qed_create(qed_ctx** out, int hip_device);
int qed_destroy(qed_ctx* ctx);
const char* qed_last_error(const qed_ctx* ctx);

/* Device allocator hook: alloc(bytes, stream, user) returns device
 * memory or NULL; free(ptr, stream, user) releases it (every block by
 * qed_destroy at the latest).  Both NULL restores the default: blocks from
 * hipMallocAsync on the context's stream, kept after release in a cache of
 * the context and handed out again to allocations of the same size class
 * on the stream that released them, returned to the pool by qed_destroy or
 * when an allocation runs out of memory.  Must be called before any device
 * allocation of the context. */
int qed_set_allocator(qed_ctx* ctx,
                      void* (*alloc)(uint64_t bytes, void* stream, void* user),
                      void (*free_fn)(void* ptr, void* stream, void* user),
                      void* user);

/* HIP stream (hipStream_t as void*) for all work of the context.  The
 * previous stream is synchronised first; cached blocks then belong to the
 * new stream. */
int qed_set_stream(qed_ctx* ctx, void* hip_stream);

/* ---------------------------------------------------------------- */
/* problem definition (Results, "The model", Eq. 1; Methods)         */
/* ---------------------------------------------------------------- */

/* Lattice Lx x Ly x Lz (sites x = (i, j, k), flat index
 * i + Lx (j + Ly k)).  Each extent must be a power of two (binary tree,
 * Methods "Tensor Networks"), with at least two sites; bc is a QED_BC_*. */
int qed_set_lattice(qed_ctx* ctx, int Lx, int Ly, int Lz, int bc);

/* Couplings of Eq. 1: hopping t, staggered mass m, electric g_e^2,
 * magnetic g_m^2 (treated as independent, as in the paper). */
int qed_set_couplings(qed_ctx* ctx, double t, double m, double g2_e, double g2_m);

/* Local chemical potentials: adds sum_x mu_x psi_x^dag psi_x to Eq. 1, the
 * large boundary or pinning potentials of the capacitor and confinement
 * set-ups (Results).  mu: host array of Lx*Ly*Lz doubles in site order
 * (copied), or NULL to remove them.  Needs qed_set_lattice first (which
 * clears them); takes effect at the next qed_build_hamiltonian.
 * QED_ERR_BAD_STATE without a lattice, QED_ERR_INVALID_ARG for non-finite
 * values. */
int qed_set_chemical_potential(qed_ctx* ctx, const double* mu);

/* Physical line (Results): with a = 1/t, g_e^2 = g^2 t, g_m^2 = 8 t / g^2,
 * so that g_e g_m = 2 sqrt(2) t.  Pure function, no context. */
int qed_physical_line(double g2, double t, double* g2_e, double* g2_m);

/* Link penalty nu sum (1 - delta_{2,L}) (Methods, penalty equation) and
 * its driven schedule (Methods, "Numerical Convergence"): n_linear sweeps
 * growing linearly from nu_max/20 to nu_max/4, then n_quadratic sweeps
 * growing quadratically to nu_max, then constant.  n_linear = n_quadratic
 * = 0 keeps nu = nu_max.  adaptive != 0: the linear phase ends early,
 * after the first linear sweep t >= 1 whose energy exceeds that of sweep
 * t - 1 by more than 1e-10 |E_t| (the energy "rises slightly"), and the
 * quadratic phase grows from the nu of that sweep to nu_max over
 * n_quadratic sweeps.  The energies looked at are those of the sweeps run
 * by this context since qed_init_state / qed_load_state (a resumed run
 * starts a new history).  QED_ERR_INVALID_ARG for nu_max < 0 or negative
 * counts. */
int qed_set_penalty(qed_ctx* ctx, double nu_max, int n_linear, int n_quadratic, int adaptive);

/* Total charge Q = N - L^3/2 (Results).  Q != 0 needs the free-flux
 * boundary; |Q| above what the boundary can carry is QED_ERR_INVALID_ARG
 * at qed_build_hamiltonian. */
int qed_set_charge_sector(qed_ctx* ctx, int Q);

/* Bond dimension chi of every internal tree leg (chi >= 1). */
int qed_set_bond_dim(qed_ctx* ctx, int chi);

/* Lanczos (Methods, step (ii)): cycles of `steps` steps with full
 * reorthogonalisation, restarted from the Ritz vector until the residual
 * is <= tol |theta| or `max_cycles` cycles ran (tol = 0: always all). */
int qed_set_lanczos(qed_ctx* ctx, int steps, int max_cycles, double tol);

/* Eigensolver precision raised sweep by sweep (Methods: the Arnoldi
 * precision is increased at every sweep): in sweep s the node updates use
 * the tolerance max(tol, tol0 * factor^s), tol from qed_set_lanczos.
 * tol0 = 0 (the default) switches the schedule off; 0 < factor < 1. */
int qed_set_lanczos_schedule(qed_ctx* ctx, double tol0, double factor);

/* Subspace expansion (Methods: single-tensor optimisation with subspace
 * expansion, which lets bond dimensions grow and symmetry sectors adapt).
 * With on != 0, every move of the isometry centre from node a to b across
 * link e is an SVD move: per charge sector, a matricised against e is
 * factored U S V^T, the largest singular values over all sectors are kept
 * (at most chi_max, 0 = the bond dimension of qed_set_bond_dim; none below
 * 1e-12 of the largest), a := U_keep and b absorbs S V^T, so the link takes
 * the kept sector sizes.  On the first move after a was updated, e is
 * first extended by up to `delta` columns per charge sector a's other legs
 * can carry (new charges included), filled with alpha |a| / |Z| Z, where
 * Z = sum_k c_k (A_k (x) B_k (x) Omega_k) a over the H_eff terms of a that
 * reach across e and Omega_k are random maps into the new columns
 * (SplitMix64 uniforms in [-1, 1) from `seed`): b does not see the new
 * columns, so the state is unchanged, and they enter the basis through
 * the truncation.  Off by default; takes effect at the next move.
 * QED_ERR_INVALID_ARG for alpha < 0 or not finite, delta < 0, chi_max < 0. */
int qed_set_expansion(qed_ctx* ctx, int on, double alpha, int delta, int chi_max, uint64_t seed);

/* GEMM arithmetic (QED_FP64 / QED_FP32 / QED_BF16) of the reduced-
 * precision paths and their refinement (Methods, "Tensor Networks", step
 * (ii) run with lower-precision products):
 *   refine = 0: Lanczos on the reduced-precision operator alone; each
 *     update's Ritz value is its energy; cycles stop at the precision's
 *     residual floor (FP32 2e-6, BF16 3.9e-3 relative);
 *   refine = 1: as 0, and the energy of each sweep (that of its last node
 *     update, the root) is an FP64 Rayleigh quotient of the Ritz vector,
 *     with an error second order in the eigenvector error;
 *   refine >= 2: FP64 residual correction at every update: the first
 *     product of every Lanczos cycle is taken with the FP64 operator, so
 *     the exact residual of the current vector enters the Krylov space and
 *     ends the update once it is below the tolerance (floors FP32 1e-8,
 *     BF16 1e-6 relative); the other products stay in reduced precision.
 *     The energy is then an FP64 Rayleigh quotient as well.
 * QED_ERR_INVALID_ARG for an unknown dtype or refine < 0. */
int qed_set_precision(qed_ctx* ctx, int gemm_dtype, int refine);

/* Build the dressed-site bases, local operators, the term list, the tree
 * and its leg sectors.  Needs lattice, couplings, charge and chi. */
int qed_build_hamiltonian(qed_ctx* ctx);

/* Local dimension of every site (int[N]). */
int qed_get_local_dims(qed_ctx* ctx, int* dims);

/* Tree shape: number of nodes, and for node n its legs as link ids
 * (site s is link s, node n's parent leg is link N + n). */
int qed_get_tree(qed_ctx* ctx, int* n_nodes, int* n_sites);
int qed_get_node_links(qed_ctx* ctx, int node, int links[3]);

/* Sectors of a link: up to `cap` (charge, size) pairs, *nsec set to the
 * full count. */
int qed_get_leg_sectors(qed_ctx* ctx, int link, int* charges, int* sizes, int cap, int* nsec);

/* ---------------------------------------------------------------- */
/* state                                                             */
/* ---------------------------------------------------------------- */

/* Seeded initial node tensors: entry i of node n is 2u - 1 with u the
 * i-th SplitMix64 uniform of stream (seed, n) (counter-based: key =
 * mix(seed ^ mix(n + 0x632BE59BD9B4E019)), word_i = mix(key + (i+1) *
 * 0x9E3779B97F4A7C15), u = (word >> 11) 2^-53). */
int qed_init_state(qed_ctx* ctx, uint64_t seed);

/* Copy one node tensor in (host, FP64, canonical flat layout of length
 * n_entries) or out.  Setting a node invalidates the environments. */
int qed_set_node(qed_ctx* ctx, int node, const double* host_blocks, int64_t n_entries);
int qed_get_node(qed_ctx* ctx, int node, double* host_blocks, int64_t n_entries);
int qed_node_size(qed_ctx* ctx, int node, int64_t* n_entries);

/* Run n sweeps (Methods: single-tensor updates from the lowest to the
 * highest layer); rep (optional, n entries) receives one record each. */
int qed_sweep(qed_ctx* ctx, int n, qed_sweep_report* rep);

/* Checkpoint / resume of the variational state (the paper's runs take
 * weeks, Methods, so a state must survive a restart).  The file holds, in
 * native byte order: magic "QEDTTNS", format version 1, lattice extents,
 * boundary, total charge, bond dimension, couplings, the sweep index (it
 * sets the penalty schedule), whether the isometry centre sits at the
 * root, the last energy, every link's (charge, size) sectors, every node's
 * FP64 blocks in canonical order, and an FNV-1a 64-bit checksum of all
 * preceding bytes.  Save writes `path`.tmp and renames it over `path`.
 * Load needs a context built (qed_build_hamiltonian) for the same lattice,
 * boundary, charge and bond dimension (couplings may differ: a warm start);
 * a state saved with the centre at the root resumes with the same
 * arithmetic as an uninterrupted run.  QED_ERR_IO for unreadable,
 * truncated or corrupt files (checked before anything changes),
 * QED_ERR_INVALID_ARG for a file of another problem. */
int qed_save_state(qed_ctx* ctx, const char* path);
int qed_load_state(qed_ctx* ctx, const char* path);

/* Failure injection for tests: overwrite the first entry of a node tensor
 * with a quiet NaN.  The next sweep reports QED_ERR_NONFINITE. */
int qed_debug_poison(qed_ctx* ctx, int node);

int qed_get_energy(qed_ctx* ctx, double* E);

/* Local observables of the current state (isometry centre moved to the
 * root): occ[N] = <psi^dag psi>_x, efield[3N] = <E_{x,mu}> (0 where the
 * link does not exist), deltaL = sum_links |<L - 2>|, rho = mean of
 * n_x = (1 - (-1)^x)/2 + (-1)^x psi^dag psi, Q = <total charge>.
 * Any output pointer may be NULL. */
int qed_get_observables(qed_ctx* ctx, double* occ, double* efield, double* deltaL,
                        double* rho, double* Q);

/* Per-site local charge and flux of the current state: charge[N] =
 * <q_x> with q_x = psi^dag psi - (1 - (-1)^x)/2 (the charge of Gauss's
 * law, Results "The model"); flux[6N] = outgoing electric flux on the six
 * half-links of each site in the order -x, -y, -z, +x, +y, +z (E_{x,mu}
 * on +mu, -E_{x-mu,mu} on -mu, the dangling flux on a free-flux boundary
 * half-link, 0 on a zero-flux one).  Gauss's law: sum_h flux = charge.
 * Any output pointer may be NULL. */
int qed_get_site_fluxes(qed_ctx* ctx, double* charge, double* flux);

/* Plane profiles along axis a in {0,1,2} (Results, "Quantum capacitor":
 * charge density and transverse field per plane).  With A the number of
 * sites of a plane orthogonal to a:
 *   qc[d] = (2/A) sum_{x in plane d} <q_x>,            d = 0 .. L_a - 1
 *   ec[d] = (2/A) sum_{x in plane d-1} <E_{x,a}>,      d = 1 .. L_a - 1
 * and ec[0], ec[L_a] the field through the lower and upper faces (the
 * dangling half-links; 0 under the zero-flux boundary).  qc holds L_a and
 * ec L_a + 1 doubles (caller-owned host arrays, either may be NULL).
 * q_x is the charge of qed_get_site_fluxes: the paper's staggered
 * psi^dag psi in the convention where the vacuum carries no charge.
 * Under zero flux, ec[d+1] - ec[d] = qc[d] whenever every link obeys the
 * rishon constraint L = 2 (the physical subspace); otherwise the
 * difference is -(2/A) times the sum of <2 - L> over the links that enter
 * plane d or lie inside it. */
int qed_get_plane_profiles(qed_ctx* ctx, int axis, double* qc, double* ec);

/* Surface charge density (Results, "Finite density", surface density
 * equation): sigma[l-1] = mean of <q_x> over the sites whose distance to
 * the closest boundary is l, l = 1 (surface) .. nshell, with nshell =
 * 1 + (min(Lx, Ly, Lz) - 1) / 2.  *nshell is written when non-NULL;
 * sigma (host, nshell doubles) may be NULL to query the count. */
int qed_get_surface_density(qed_ctx* ctx, double* sigma, int* nshell);

/* Pin static charges with large local chemical potentials (Results,
 * "Confinement properties" and "Quantum capacitor"): for each i, site
 * sites[i] gets mu += -lambda when charges[i] + parity = 1 (filled) and
 * +lambda when it is 0 (empty); +1 needs an even site, -1 an odd site, 0
 * pins the site's vacuum occupation.  Adds to the potentials already set
 * (qed_set_chemical_potential; qed_set_lattice clears both); takes effect
 * at the next qed_build_hamiltonian.  The pinning energy is part of the
 * ground-state energy, so V(r) = E(r) - E_0 carries the r-independent
 * constant -lambda per pinned pair.  QED_ERR_INVALID_ARG for a site out of
 * range or pinned twice, a charge the site's parity cannot hold, or
 * lambda not finite and positive; QED_ERR_BAD_STATE without a lattice. */
int qed_pin_charges(qed_ctx* ctx, int n, const int* sites, const int* charges, double lambda);

/* Cumulative counters of the context.  matvec_flops / matvecs: algorithmic
 * work of every H_eff application (sweeps and node-level objects).
 * With profiling on, the block-GEMM and fused launches of every H_eff
 * application are timed with HIP events on the context's stream: one
 * event pair brackets an application's GEMM launches (issued back to back),
 * or, with QEDTTN_TRACE set or fused stages in the plan, each launch gets
 * its own pair.  gemm_launches counts the launches, gemm_ms sums the event
 * intervals and gemm_flops the algorithmic flops of those launches;
 * fused_launches, fused_ms and fused_flops count the fused kernel's
 * launches alone. */
typedef struct {
    double matvec_flops;
    long long matvecs;
    long long gemm_launches;
    double gemm_ms;
    double gemm_flops;
    long long fused_launches;
    double fused_ms;
    double fused_flops;
} qed_stats;

/* Profiling switch (0/1) for the H_eff block-GEMM launches; resets the
 * GEMM counters.  Synchronises the stream when stats are read. */
int qed_set_profiling(qed_ctx* ctx, int on);
int qed_get_stats(qed_ctx* ctx, qed_stats* out);

/* ---------------------------------------------------------------- */
/* block tables (pure host integer work, bit-exact contract)         */
/* ---------------------------------------------------------------- */

/* Allowed blocks of a three-leg tensor with the given flux.  triples
 * (3*nblk ints: sector indices l, r, p) and offs (nblk+1 int64) may be
 * NULL to query *nblk first; cap is the capacity in blocks. */
int qed_node_blocks(const int* ch_l, const int* n_l, int s_l,
                    const int* ch_r, const int* n_r, int s_r,
                    const int* ch_p, const int* n_p, int s_p,
                    int flux, int cap, int* nblk, int* triples, int64_t* offs);

/* ---------------------------------------------------------------- */
/* node-level effective Hamiltonian (Methods, steps (i)-(ii))         */
/* ---------------------------------------------------------------- */

/* One term c * A (x) B (x) C.  op[i] is a device FP64 block-sparse leg
 * operator (layout above) for leg i (0 = l, 1 = r, 2 = p) with charge
 * shift shift[i], or NULL for the identity.  shift_l + shift_r must
 * equal shift_p. */
typedef struct {
    double coef;
    const double* op[3];
    int shift[3];
} qed_term;

/* Build H_eff = sum_k terms[k] on a node with the given legs, in the
 * context's GEMM precision.  Operators are copied (converted) at create
 * time; the caller keeps ownership of its buffers. */
int qed_heff_create(qed_ctx* ctx,
                    const int* ch_l, const int* n_l, int s_l,
                    const int* ch_r, const int* n_r, int s_r,
                    const int* ch_p, const int* n_p, int s_p,
                    int K, const qed_term* terms, qed_heff** out);
int qed_heff_destroy(qed_heff* h);

/* y = H_eff x on device FP64 flat vectors of length *size (x, y must not
 * alias). */
int qed_heff_size(qed_heff* h, int64_t* size);
int qed_heff_matvec(qed_heff* h, const double* x, double* y);

/* Size of the scratch area of qed_heff_matvec_noalloc, per GPU. */
#define QED_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * y = H_eff x as qed_heff_matvec (same plan and kernels, same result),
 * with the stage intermediates held in a fixed scratch area of
 * QED_NOALLOC_SCRATCH_BYTES that the library keeps on every GPU it runs
 * on from load to process exit, instead of the handle's own workspace.
 * The call allocates nothing: no hipMalloc, hipFree or allocating library
 * routine (reduced-precision handles use the staging buffers that
 * qed_heff_create made).  x, y: device FP64, length qed_heff_size,
 * distinct; work is enqueued on the context's stream.
 * Errors: QED_ERR_INVALID_ARG, with nothing launched, when the handle's
 * stage workspace exceeds the scratch size (the message gives both);
 * QED_ERR_HIP when the scratch address of the device could not be looked
 * up at qed_create.  Every call on one GPU shares that GPU's scratch, so
 * calls whose work overlaps on the device (several streams, threads or
 * contexts) race on it; the scratch keeps the last call's contents, and
 * no call reads a scratch element before writing it.  No profiling
 * events are recorded for this call. */
int qed_heff_matvec_noalloc(qed_heff* h, const double* x, double* y);

/* Lanczos for the lowest eigenpair started from x (device FP64); x is
 * overwritten by the normalised Ritz vector; *eval receives theta and
 * *resid (may be NULL) the residual estimate.  `steps` per cycle, cycles
 * and tolerance as set by qed_set_lanczos (steps <= 0: context value). */
int qed_heff_lanczos(qed_heff* h, double* x_inout, int steps, double* eval, double* resid);

/* Algorithmic work of one matvec: flops (identity factors and skipped
 * dense work not counted) and the bytes of x, y and the non-identity
 * operator blocks in the GEMM dtype. */
int qed_heff_flops(qed_heff* h, double* flops, double* bytes);

/* Reverse mode of y = H_eff x (the effective Hamiltonian of Methods step
 * (i) as a differentiable function of the node tensor, of every factor
 * and of every coefficient), given the cotangent ybar:
 *   xbar = sum_k c_k (A_k^T (x) B_k^T (x) C_k^T) ybar,
 *   opbar[3k+e] = d<ybar, y>/d(factor e of term k), in that factor's
 *                 operator layout (shift unchanged),
 *   coefbar[k]  = <ybar, A_k (x) B_k (x) C_k x>.
 * x, ybar: device FP64 (length qed_heff_size); xbar: device FP64 or NULL;
 * opbar: NULL or 3K device FP64 pointers (NULL entries skipped; entries
 * for identity factors ignored); coefbar: host double[K] or NULL.  The
 * contractions run in the context's GEMM precision; intermediates are
 * recomputed, nothing from a forward call is stored.  The first call
 * builds the transposed factors and the contraction schedule. */
int qed_heff_matvec_adjoint(qed_heff* h, const double* x, const double* ybar, double* xbar,
                            double* const* opbar, double* coefbar);

/* Algorithmic flops of one adjoint call: the transposed-factor matvec for
 * xbar, and the mode products plus two-tensor contractions for all factor
 * gradients (the coefficient dot products are not counted).  Builds the
 * adjoint schedule if no adjoint call has yet. */
int qed_heff_adjoint_flops(qed_heff* h, double* xbar_flops, double* grad_flops);

/* ---------------------------------------------------------------- */
/* batched node updates                                              */
/* ---------------------------------------------------------------- */

/* One node of a batch: its three legs and its terms (as in
 * qed_heff_create; operators are copied at create time). */
typedef struct {
    const int* ch[3];
    const int* n[3];
    int nsec[3];
    int K;
    const qed_term* terms;
} qed_heff_desc;

/* Many independent node-level effective Hamiltonians in one object: every
 * contraction stage of all nodes is one grouped block-GEMM launch, and the
 * Lanczos recurrences of all nodes advance together (one per node).  The
 * batch works on the concatenation of the nodes' flat vectors (node i at
 * offset offs[i]). */
int qed_heff_batch_create(qed_ctx* ctx, int nnodes, const qed_heff_desc* nodes,
                          qed_heff_batch** out);
int qed_heff_batch_destroy(qed_heff_batch* b);

/* Total length of the concatenated vector and (optional, nnodes + 1)
 * per-node offsets. */
int qed_heff_batch_size(qed_heff_batch* b, int64_t* total, int64_t* offs);

/* y = blockdiag(H_eff,i) x on device FP64 concatenated vectors. */
int qed_heff_batch_matvec(qed_heff_batch* b, const double* x, double* y);

/* Lowest eigenpair of every node: x (device FP64, concatenated) holds the
 * start vectors and receives the normalised Ritz vectors; evals[nnodes]
 * and resids[nnodes] (may be NULL) receive theta and the residual
 * estimates.  use_graph != 0 replays a HIP graph of one whole cycle
 * (captured on first use for this step count).  Cycles and tolerance as
 * set by qed_set_lanczos (a cycle ends for all nodes when every node has
 * converged).  The recurrence runs in FP64; with FP32 GEMMs and at most 31
 * steps the Krylov basis is stored in FP32 (the matvec reads its input
 * from it; environment QEDTTN_LZ_BASIS=fp64 keeps it in FP64). */
int qed_heff_batch_lanczos(qed_heff_batch* b, double* x_inout, int steps, double* evals,
                           double* resids, int use_graph);

/* Algorithmic flops and bytes of one batched matvec. */
int qed_heff_batch_flops(qed_heff_batch* b, double* flops, double* bytes);

/* Autotuner: from now on, node-level and batched H_eff objects time every
 * (workgroup tile shape, operand pipeline) pair each GEMM stage allows -
 * three tile shapes; the register-staged loop, the flat product pipeline
 * and, for FP32, the LDS-DMA ring - and keep the fastest.
 * Decisions are cached per stage signature and, if cache_path is not
 * NULL, loaded from and saved to that text file.  cache_path = "" turns
 * tuning off. */
int qed_autotune(qed_ctx* ctx, const char* cache_path);

#ifdef __cplusplus
}
#endif

#endif /* QEDTTN_H */
