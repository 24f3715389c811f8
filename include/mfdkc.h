/*
 * mfdkc: kernel-compensated mimetic finite differences for the Maxwell
 * eigenproblem in photonic crystals (arXiv 2503.19379), on MI355X (gfx950).
 *
 * C ABI.  Plain pointers and sizes only.  Every function returns MFD_OK (0) or
 * a negative mfd_status; no C++ exception crosses this boundary, and
 * mfd_last_error() gives a thread-local detail string for the last failure.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid.  The periodic cube [0, L]^3 is cut into N^3 cells of side h = L / N
 *   (Section 4.1.1).  A grid function is stored [z][y][x], x fastest: linear
 *   index x + N (y + N z).  This is the order implied by the Kronecker form
 *   K_1 = I (x) I (x) D_1 / h of eq. (blocks).
 * Fields.  The unknown H lives on cell faces F_h (eq. (DoFs_grid)).  One
 *   field is 3 components x N^3 complex values, stored [comp][z][y][x].  A
 *   block of nb fields is stored [band][comp][z][y][x], i.e. column-major
 *   n x nb with n = 3 N^3.  Complex values are interleaved (re, im):
 *   MFD_C128 = two doubles, MFD_C64 = two floats.
 * Bloch vector.  k = (k_x, k_y, k_z) is Cartesian, in units of 1/L; it is
 *   the shift alpha of the discrete operators (Section 4.1.2).
 * Operator.  op(k) = A M_0 A' + gamma(k) B'B + c(k) I with A = curl_alpha,
 *   B = div_alpha (eq. (discrete_2nd_block)), M_0 = diag(mu) on edges from
 *   eps^-1 (Section 4.4), gamma(k) the penalty number (eq. (pnt_number)) and
 *   c(k) the shift of Remark 5.1.  Readings of the paper used here:
 *     mu on an edge = 4 / (sum of eps over the 4 cells sharing the edge);
 *     gamma(k) = 2 max{ N / (2 pi), (2 pi / (L max(|k|, k_b)))^2 }, i.e. the
 *       rule of eq. (pnt_number) in the paper's units of lattice constant
 *       2 pi, with |k| clamped below at k_b = pi / (2L) (unclamped, FP64
 *       rounding of gamma B'B x exceeds a 1e-8 relative residual near
 *       Gamma), unless set by mfd_set_gamma;
 *     c(k) = (pi / L)^2 if |k| < k_b, else 0 (Remark 5.1, used in the ball
 *       around Gamma where A A' + gamma B'B is singular or nearly so).
 *   Eigenvalues reported by mfd_bands have c(k) subtracted.  Residuals are
 *   relative to |lambda| + c(k).
 * Streams.  Every call is ordered on `stream` (a hipStream_t passed as
 *   void*; NULL = the null stream).  mfd_op_apply and mfd_precond_solve are
 *   asynchronous to the host; mfd_bands returns once evals are on the host.
 * Ownership.  The caller owns every buffer passed in.  The library owns the
 *   context (device copies of M_0, FFT twiddles, solver workspace), freed by
 *   mfd_destroy.  A context is not thread safe: use one per host thread.
 */
#ifndef MFDKC_H
#define MFDKC_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mfd_ctx mfd_ctx;

/* MFD_C64_F64 (mfd_op_apply only): MFD_C64 storage, FP64 arithmetic with
 * the FP64 M_0, the form the mixed-precision solver applies to its
 * FP32-stored blocks. */
typedef enum { MFD_C64 = 1, MFD_C128 = 2, MFD_C64_F64 = 3 } mfd_dtype;

typedef enum {
    MFD_OK = 0,
    MFD_EINVAL = -1,        /* bad argument (null pointer, size, non-finite or non-positive eps, aliasing) */
    MFD_ENOMEM = -2,        /* device allocation failed */
    MFD_EDEVICE = -3,       /* a HIP call or kernel launch failed */
    MFD_ENOTCONV = -4,      /* max_iter reached; evals/stats hold the best values found */
    MFD_ESPURIOUS = -5,     /* Alg 4.1 still flags a band after max_gamma_doublings */
    MFD_EUNSUPPORTED = -6   /* grid size or stencil order this build does not handle */
} mfd_status;

/* Options of mfd_bands.  Zero-initialise, then set what you need;
 * mfd_default_opts fills in the defaults. */
typedef struct {
    int max_iter;             /* LOBPCG iterations per k-point (default 400) */
    int precision;            /* 0: FP64 throughout; 1: mixed FP32 corrections + FP64 refinement */
    int warm_start;           /* 0: random start at every k (seed); 1: previous k's vectors;
                                 2: learned: previous k's vectors plus a block proposed by a small
                                 network trained along the path (see mfd_mlp_*), once 4 training
                                 pairs exist; the first Rayleigh-Ritz step uses both */
    unsigned long long seed;  /* random start blocks */
    int max_gamma_doublings;  /* Alg 4.1 restarts (default 4) */
    int guard;                /* extra block columns beyond nbands (default 2); they also hold
                                 compensation modes that Alg 4.1 flags and discards */
    int streams;              /* k-path segments (mfd_bands) or crystals (mfd_bands_batch) solved
                                 concurrently, each on its own stream and host thread (default 4,
                                 at most 16).  The streams run side by side only with as many
                                 hardware queues: set GPU_MAX_HW_QUEUES >= streams before the
                                 process first uses HIP (HIP's default is 4) */
    const void* x0;           /* optional device c128 start block [nbands][3][N][N][N] for the first
                                 k-point (NULL: random); a column numerically dependent on the ones
                                 before it (squared distance to their span below 1e-10 of its squared
                                 norm, or a zero column) is replaced by seeded random values */
    int stall_window;         /* iterations without a halving of the largest residual after
                                 which precision 1 continues the k-point in FP64 (default 40,
                                 0 = never); FP64 restarts its conjugate directions from the
                                 current vectors after max(stall_window, 40) such iterations */
    int learn_steps;          /* warm_start 2: Adam steps over the replay buffer after each new
                                 training pair (default 30; 0 = the untrained network, which
                                 proposes the previous step's combination unchanged) */
    float learn_rate;         /* warm_start 2: Adam learning rate (default 1e-3) */
    int autotune;             /* 1 (default): on the first call for a context and block shape, time
                                 candidate launch shapes of the Gram, update, stencil and FFT kernels
                                 and keep the fastest (see mfd_tuning); 0: built-in shapes */
    int precond;              /* preconditioner solve: 0 (default) the FFT solve of Alg 5.1
                                 (mfd_precond_solve); 1 the multigrid solve of Section 5.3
                                 (mfd_precond_solve_mg: cubic contexts of order 2 whose grid
                                 mfd_mg_supported accepts; MFD_EUNSUPPORTED otherwise) */
    int mg_cycles;            /* precond 1: V-cycles per scalar solve (default 2) */
    int mg_smooth;            /* precond 1: pre- and post-smoothing steps per level (default 2) */
    int mg_sweeps;            /* precond 1: Jacobi sweeps per ILU factor in a smoothing step (default 2) */
    int graph;                /* 1: from the third iteration of a k-point on, run the iterations in
                                 chunks of 2 to 8 replayed from a HIP graph captured once per basis
                                 shape (two LOBPCG iterations per graph), with the host reading the
                                 residuals only between chunks; the active set is frozen within a
                                 chunk.  0 (default): the host steps every iteration */
    int cold_start;           /* start block of a segment's first k-point (without x0): 0 (default)
                                 seeded random; 1 the lowest transverse plane waves at k, ordered
                                 by |k + G| (the eigenvectors of the operator with a uniform
                                 medium), plus 0.1 of the seeded random block */
    int balance;              /* mfd_bands: 1 = a stream whose k-path segment is done takes the
                                 second half of the k-points still ahead of the busiest other
                                 segment (at least 2 beyond the one it is solving), starting
                                 it as a segment of its own (cold start); the cut points then
                                 depend on timing, so bands agree between runs to the
                                 tolerance, not bit for bit.  Not with warm_start 2.
                                 0 (default): fixed segments of equal length */
    int hard_lock;            /* 1: once at most 8 bands of a k-point still iterate, the converged
                                 ones are locked: their vectors stay as they are and leave the
                                 Rayleigh-Ritz basis, the new search directions are made
                                 orthogonal to them, and the block update touches only the bands
                                 still iterating (a locked band whose fresh residual misses the
                                 tolerance iterates again).  0 (default): soft locking only */
} mfd_opts;

typedef struct {
    int iters;                /* LOBPCG iterations, summed over gamma restarts */
    int gamma_doublings;      /* Alg 4.1 restarts taken */
    double gamma;             /* penalty number used for the returned bands */
    double max_rel_resid;     /* max_i |op x_i - theta_i x_i| / (theta_i |x_i|), FP64 operator */
    int spurious;             /* bands still flagged by Alg 4.1 among those returned */
    int discarded;            /* flagged bands skipped in favour of the next physical ones */
    int used_fallback;        /* warm_start 2: the previous-k start was used alone, because no
                                 proposal was available (fewer than 4 training pairs, or dependent
                                 history blocks) or because the proposal's Ritz-value sum was not
                                 below the previous-k block's */
    int fp64_fallback;        /* precision 1 only: the FP32-stored directions stalled (no halving
                                 of the residual in stall_window iterations) and the k-point was
                                 finished in FP64 from the current block */
    float ms;                 /* wall time of this k-point */
    int rejected_steps;       /* Rayleigh-Ritz steps rejected: a step whose Ritz values are not the
                                 Rayleigh quotients of its vectors under a fresh operator application
                                 (a nearly dependent search direction amplified the rounding of its
                                 Gram entries) is undone, A X recomputed and P restarted; mixed
                                 precision then continues in FP64 (unless stall_window is 0) */
    int host_syncs;           /* host synchronisations with the solve's stream for this k-point */
    int segment_start;        /* 1: the k-point began a segment (x0, plane-wave or random start);
                                 0: it started from the previous k-point's vectors */
} mfd_kstats;

void mfd_default_opts(mfd_opts* opts);

/* Build a context for one crystal (Section 4.4: M_0 from eps).
 * N: cells per axis, 4 <= N <= 150, with an FFT plan for N (N = 2^a 3^b 5^c
 *    supported by this build: 8, 10, 12, 16, 20, 24, 32, 40, 48, 64, 80, 96,
 *    100, 120, 128, 150; see mfd_supported_n).
 * L: cell side (> 0).  order: stencil order 2, 4, 6 or 8 (Section 4.1.3,
 *    eq. (2kfdm), Table FD_1D with k = order / 2; the sixth-order c_1 is read as
 *    75/64, the value the stencil's consistency requires).  Order 2 uses the
 *    fused single-pass stencil; higher orders use a two-pass operator with a
 *    scratch buffer owned by the context (and one per band-solve workspace).
 * eps_cells: host, N^3 doubles, [z][y][x], finite and > 0 (cell permittivity).
 * Errors: MFD_EINVAL, MFD_EUNSUPPORTED, MFD_ENOMEM, MFD_EDEVICE. */
int mfd_build(int N, double L, int order, const double* eps_cells, void* stream, mfd_ctx** out);

/* As mfd_build, with M_0 given directly: mu_edges (host, 3 N^3 doubles,
 * [comp][z][y][x], finite and > 0) is the diagonal of M_0 on the edges, edge
 * e_1 at ((x + 1/2) h, y h, z h), e_2 at (x h, (y + 1/2) h, z h), e_3 at
 * (x h, y h, (z + 1/2) h).  Section 6.2 builds M_0 this way for its cubic
 * lattices: eps_1^-1 on the edges inside the material, eps_0^-1 outside.
 * Errors as mfd_build. */
int mfd_build_mu(int N, double L, int order, const double* mu_edges, void* stream, mfd_ctx** out);

/* As mfd_build, on a general lattice (Section 2, eq. (coordinate_change);
 * Section 4.2, "Matrix representation on general lattices").
 * lattice: host, 9 doubles, row-major 3 x 3 matrix A whose columns are the
 *    primitive vectors a_1, a_2, a_3 (Cartesian; lattice[3 r + c] = component r
 *    of a_{c+1}), linearly independent.  The grid is the unit cube of
 *    y = A^-1 x with N cells per axis; eps_cells ([z][y][x] as for mfd_build)
 *    holds the permittivity of the cell centred at y = ((x+1/2), (y+1/2),
 *    (z+1/2)) / N.  Every derivative becomes D^_i = sum_j b_ji K_j + i L_i with
 *    b = A^-1, K_j the difference along grid axis j and L_i the unchanged
 *    average along grid axis i (alpha = the Cartesian k).
 * Wave vectors passed to the other calls stay Cartesian (units 1/length of A).
 * The penalty and shift rules use L = |det A|^(1/3) in place of the cell side.
 * Order 2 uses a fused single-pass kernel (z-marching tiles in LDS); orders
 * 4-8 the two-pass operator (scratch owned by the context).
 * Errors: MFD_EINVAL also for a NULL, non-finite or singular lattice; others
 * as mfd_build. */
int mfd_build_lattice(int N, const double* lattice, int order, const double* eps_cells, void* stream,
                      mfd_ctx** out);

/* As mfd_build_lattice, with M_0 given on the edges of the unit-cube grid
 * (mu_edges as for mfd_build_mu, edge e_1 at y = ((x + 1/2), y, z) / N and so
 * on).  Section 6.3 sets M_0 this way for its BCC and FCC cells. */
int mfd_build_lattice_mu(int N, const double* lattice, int order, const double* mu_edges, void* stream,
                         mfd_ctx** out);

/* Band-gap ratio of Section 6.2 from a computed band structure (host only):
 * for each pair of consecutive bands j, j + 1 (1-based j), omega_low = the
 * largest omega of band j over the nk k-points, omega_up = the smallest of
 * band j + 1, ratio = (omega_up - omega_low) / ((omega_up + omega_low) / 2),
 * with omega = sqrt(lambda) (lambda below zero, roundoff at Gamma, counts as
 * zero).  Returns the largest ratio over the pairs in *ratio and its lower
 * band j in *below; a ratio <= 0 means no gap.  evals: host nk x nbands (as
 * mfd_bands writes it), finite; nk >= 1, nbands >= 2.
 * kpts: host nk x 3 (the k-points of evals), or NULL.  At k = 0 mfd_bands
 * returns the three constant fields as bands 1-3; two of them continue the
 * two lowest bands as k -> 0 and the third is a static mode through which no
 * band passes.  With kpts given, a row with k exactly 0 skips that third
 * zero: its band j >= 3 is the returned value j + 1, and it has no value for
 * the last band.  With NULL, every row is taken as returned.
 * Errors: MFD_EINVAL for NULL outputs, bad sizes, non-finite values, or when
 * no pair gives a ratio (a lone k = 0 row with nbands = 3: 0/0 for bands
 * 1-2, no value of band 3). */
int mfd_gap_ratio(int nk, int nbands, const double* kpts, const double* evals, double* ratio, int* below);

/* Largest nbands + guard that mfd_bands and mfd_bands_batch accept. */
int mfd_max_block(void);

/* 1 if this build has an FFT plan and stencil for grid size N, else 0. */
int mfd_supported_n(int N);

/* Override the penalty number (gamma > 0), or restore the rule (gamma <= 0). */
int mfd_set_gamma(mfd_ctx* ctx, double gamma);

/* gamma(k) and c(k) this context uses at k (host, no device work). */
int mfd_gamma_shift(const mfd_ctx* ctx, const double k[3], double* gamma, double* shift);

/* Y = op(k) X for nb fields (eq. (Ker_comp) plus the shift c(k)).
 * X, Y: device, [nb][3][N][N][N] interleaved complex of `dtype`; must not
 * overlap.  FP32 (MFD_C64) uses an FP32 copy of M_0; MFD_C64_F64 reads and
 * writes FP32 and computes in FP64. */
int mfd_op_apply(mfd_ctx* ctx, const double k[3], int nb, int dtype, const void* X, void* Y,
                 void* stream);

/* T = (P + c(k) I)^-1 R for nb fields, with P = A A' + gamma B'B the
 * preconditioner of Section 5.1 eq. (penalised_marix), solved as in Alg 5.1:
 * forward FFT along each axis, the 3 x 3 symbol solve at every frequency
 * (closed-form rank-one inverse: P_hat = s I + (gamma - 1) conj(d) d^T),
 * inverse FFT along each axis.  R and T may be the same buffer.
 * Both dtypes take every N that mfd_supported_n accepts.  The x-y plane pass
 * holds a whole plane in LDS where it fits (MFD_C128 up to N = 96, MFD_C64 up
 * to 128); above that it runs as an x pass and a y pass, two more reads and
 * writes of the block. */
int mfd_precond_solve(mfd_ctx* ctx, const double k[3], int nb, int dtype, const void* R, void* T,
                      void* stream);

/* The same system as mfd_precond_solve, (P + c(k) I) T = R, solved by
 * multigrid (Section 5.3, Alg 5.2).  The distributive form of Section 5.3 is
 * used: with L_k = B B' the cell Laplacian of Cor 4.4 (A A' + B'B =
 * diag(L_k, L_k, L_k), B A = 0), the exact solution is y = (L_k + c)^-1 R per
 * component, q = -(gamma L_k + c)^-1 (gamma - 1) B y, T = y + B' q; each scalar
 * solve is replaced by `cycles` V-cycles from a zero guess on the grids N,
 * N/2, ... (rediscretised, halving while N is even and above 4; exact solve on
 * the coarsest grid), with `smooth` pre- and post-smoothing steps of the
 * ILU(0) smoother whose triangular factors are inverted approximately by
 * `sweeps` Jacobi sweeps (ILU-SAIT), cell-centred full-weighting restriction
 * and trilinear prolongation.  cycles >= 1, smooth >= 0, sweeps >= 0.
 * R, T: device [nb][3][N][N][N] of `dtype` (MFD_C64 or MFD_C128; arithmetic is
 * FP64 either way); T may be R.  Work space (about 7 x 3 nb FP64 grids) is
 * owned by the context and grows on demand.
 * MFD_EUNSUPPORTED unless the context is cubic, of order 2, and
 * mfd_mg_supported(N). */
int mfd_precond_solve_mg(mfd_ctx* ctx, const double k[3], int nb, int dtype, int cycles, int smooth, int sweeps,
                         const void* R, void* T, void* stream);

/* 1 if the multigrid hierarchy of grid size N (halving while even and above
 * 4) ends on a grid of at most 5 cells per axis, e.g. N = 8, 16, 24, 32, 48,
 * 64, 80, 96; else 0 (e.g. N = 100, 120). */
int mfd_mg_supported(int N);

/* lambda_re of Alg 4.1: out[i] = |M_0^(1/2) A' x_i|^2 / |x_i|^2 for nb c128
 * fields X (device).  out: host, nb doubles. */
int mfd_lambda_re(mfd_ctx* ctx, const double k[3], int nb, const void* X, double* out, void* stream);

/* mfd_lambda_re for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same values, computed by the same kernels, with the partial sums kept in
 * a static device array of the library (about 130 KB per GPU, held until the
 * process ends) instead of buffers allocated per call.
 * X: device c128 [nb][3][N][N][N]; out: device, nb doubles (written by a
 * kernel: the call is asynchronous, stream-ordered on `stream`, and calls no
 * hipMalloc, hipFree or host synchronisation).  nb <= 64 (MFD_EINVAL above).
 * The context must belong to the current device.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams,
 * other host threads) race and must be ordered by the caller. */
int mfd_lambda_re_static(mfd_ctx* ctx, const double k[3], int nb, const void* X, double* out, void* stream);

/* Lowest nbands physical eigenpairs at each of nk Bloch vectors: LOBPCG
 * (Section 5.1) on nbands + guard columns preconditioned by
 * mfd_precond_solve, then the recompute check of Alg 4.1: bands it flags as
 * spurious are discarded when enough physical ones remain among the
 * nbands + guard, otherwise gamma is doubled and the solve repeated.
 * The k-points are cut into opts->streams contiguous segments solved
 * concurrently; inside a segment each k-point starts from the previous one's
 * vectors (warm_start = 1).
 * kpts: host nk x 3.  tol: relative residual target (see mfd_kstats).
 * nbands + opts->guard <= mfd_max_block() = 22 (the basis of 3 (nbands +
 * guard) columns, at most 66, is what the one-workgroup Rayleigh-Ritz step
 * holds in LDS); MFD_EUNSUPPORTED otherwise.  20 bands take guard <= 2.
 * FP64 iterations on grids above N = 96 apply the preconditioner to an FP32
 * copy of the search directions (the FP64 plane FFT does not fit in LDS). 
 * evals: host nk x nbands, ascending.  evecs: device c128
 * [nk][nbands][3][N][N][N] or NULL.  stats: host nk entries or NULL.
 * Returns MFD_ENOTCONV / MFD_ESPURIOUS after filling evals and stats. */
int mfd_bands(mfd_ctx* ctx, int nk, const double* kpts, int nbands, double tol,
              const mfd_opts* opts, double* evals, void* evecs, mfd_kstats* stats, void* stream);

/* Many crystals in one call (uneven grids allowed): crystal c has context
 * ctxs[c] (distinct), nk[c] k-points kpts[c] (host nk[c] x 3) and writes
 * evals[c] (host nk[c] x nbands) and stats[c] (host nk[c], or stats = NULL).
 * Crystals are distributed over opts->streams concurrent workers; each
 * crystal's k-path is solved in order with warm starts.  opts->x0 must be NULL.
 * Same return codes as mfd_bands. */
int mfd_bands_batch(int ncrys, mfd_ctx* const* ctxs, const int* nk, const double* const* kpts, int nbands,
                    double tol, const mfd_opts* opts, double* const* evals, mfd_kstats* const* stats,
                    void* stream);

/* Per-kernel timing of mfd_bands with HIP events recorded on the solve's
 * stream around each launch group.  mfd_profile(ctx, 1) clears the counters
 * and starts recording, (ctx, 0) stops.  mfd_profile_read fills 6 entries per
 * array, by category: 0 stencil (mfd_op_apply kernel), 1 FFT preconditioner
 * (three kernels), 2 Gram product (the tile kernel alone), 3 Rayleigh-Ritz,
 * 4 block update (the update kernel alone), 5 the fixed-order sums of the
 * Gram tiles and of the update's column norms.  ms: total event time, count:
 * launches, bytes: algorithmic HBM bytes (each block read or written once);
 * for the Gram product (category 2) its flops instead, 8 n K (K + 1) for the
 * launch's basis of K columns (two Hermitian K x K products, upper halves). */
int mfd_profile(mfd_ctx* ctx, int enable);
int mfd_profile_read(mfd_ctx* ctx, double* ms, long long* count, double* bytes);

void mfd_destroy(mfd_ctx* ctx);

const char* mfd_strerror(int status);
const char* mfd_last_error(void);

/* Launch shapes the autotuner chose for ctx (out: 5 ints): out[0] Gram
 * workgroups, out[1] update workgroups, out[2] stencil workgroup target,
 * out[3] FFT plan: the z-pass x run (0 built-in), or -1 for the
 * register-resident passes (FP32 storage, cubic order 2, N = 16, 32 or 64),
 * out[4] update form: 0 one wave per 16-row strip,
 * 16 or 32 rows per workgroup block.
 * Returns 1 when tuned or pinned, 0 when not yet (out holds zeros), MFD_EINVAL
 * on NULL. */
int mfd_tuning(const mfd_ctx* ctx, int* out);

/* Pin the launch shapes (in: 5 ints, laid out as mfd_tuning reports them) for
 * every later solve on ctx, whatever its block shape; the autotuner then does
 * not run on ctx.  Each value must be one of the autotuner's candidates:
 * Gram workgroups {128, 256, 512, 1024}, update workgroups {256, 512, 1024,
 * 2048}, stencil workgroups {512, 1024, 2048, 4096}, FFT plan {0 (built-in),
 * 4, 8, 16 dividing N, -1 where the register-resident passes apply}, update
 * form {0, 16, 32}; else MFD_EINVAL and nothing
 * changes.  A workgroup count beyond what a workspace's partial buffers hold
 * keeps the built-in one for that workspace.  in = NULL clears the pin and any
 * tuning: the built-in shapes apply until the autotuner runs again.
 * Returns MFD_OK, or MFD_EINVAL (NULL ctx, value outside the candidates). */
int mfd_set_tuning(mfd_ctx* ctx, const int* in);

/* ---------------------------------------------------------------------------
 * Learned warm start: the network's kernels.  A small multilayer perceptron
 * x -> gelu(W1 x + b1) -> ... (nlayers hidden layers of width nhidden) ->
 * W_out h + b_out, gelu(z) = z Phi(z) with the exact normal CDF, trained with
 * mean-squared-error loss and Adam.  Parameters are one flat FP32 vector: per
 * layer W (out x in, row-major) then b.  With bf16_weights the products read a
 * bfloat16 copy of the weights (round to nearest even after every step) and
 * accumulate in FP32; otherwise they read the FP32 parameters.  These
 * functions serve the band solver's warm_start = 2 and direct checks of the
 * network; the paper has no learned component.
 * ------------------------------------------------------------------------- */
typedef struct mfd_mlp mfd_mlp;

/* Glorot-uniform hidden layers (seeded), zero output layer.  max_batch bounds
 * the batch of every later call.  MFD_EINVAL on non-positive sizes. */
int mfd_mlp_create(int nin, int nhidden, int nlayers, int nout, int max_batch, int bf16_weights,
                   unsigned long long seed, mfd_mlp** out);
long long mfd_mlp_num_params(const mfd_mlp* net);
/* host FP32 parameters in and out; set_params also clears Adam's moments and step count */
int mfd_mlp_set_params(mfd_mlp* net, const float* params);
int mfd_mlp_get_params(mfd_mlp* net, float* params);
/* Y (device, batch x nout FP32, row-major) = network(X) (device, batch x nin). */
int mfd_mlp_forward(mfd_mlp* net, int batch, const float* X, float* Y, void* stream);
/* loss = mean over batch and outputs of (network(X) - T)^2 (host, blocking);
 * the gradient stays in the network for mfd_mlp_adam_step and is copied to
 * grad (device, nparams FP32) when grad is not NULL. */
int mfd_mlp_loss_grad(mfd_mlp* net, int batch, const float* X, const float* T, double* loss, float* grad,
                      void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) from the last gradient. */
int mfd_mlp_adam_step(mfd_mlp* net, float lr, void* stream);
void mfd_mlp_destroy(mfd_mlp* net);

/* Training target of the warm start from three converged blocks Xa = X_{j-1},
 * Xb = X_j, Xc = X_{j+1} (device c128, each n x mb column-major, mb <= 22):
 * C (device c128, 2mb x mb row-major) = Y^H Xc Q with Y = [Xb Xa] R^-1
 * (R^H R the Gram matrix of [Xb Xa]) and Q the unitary polar factor of
 * Xc^H Xb; Rinv (device c128, 2mb x 2mb row-major, or NULL) = R'^-1 for the
 * Gram matrix R'^H R' of [Xc Q, Xb] (the basis of the next proposal, with Xc
 * aligned to Xb).  Blocking.  MFD_ENOTCONV when [Xb Xa] or
 * [Xc Xb] is numerically rank deficient (relative pivot below 1e-10). */
int mfd_warm_target(long long n, int mb, const void* Xa, const void* Xb, const void* Xc, void* C, void* Rinv,
                    void* stream);

/* Input row of the warm start's network for the step k_j -> k_next (the
 * learned warm start is not in the paper): row (device FP32, 6 + 2mb + 4mb^2
 * floats) = [k_next L/pi (3), (k_next - k_prev) L/pi (3), lam_j / (2pi/L)^2
 * (mb), lam_jm1 / (2pi/L)^2 (mb), C as (re, im) pairs in row-major order],
 * with k_prev = k_j and C (device c128, 2mb x mb row-major) the training
 * target C*_j of the previous step (mfd_warm_target).  k_prev, k_next (3
 * doubles) and lam_j, lam_jm1 (mb doubles) are host arrays.  mb <= 22.
 * Blocking; MFD_EINVAL on NULL pointers or bad sizes. */
int mfd_warm_features(double L, int mb, const double* k_prev, const double* k_next, const double* lam_j,
                      const double* lam_jm1, const void* C, float* row, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MFDKC_H */
