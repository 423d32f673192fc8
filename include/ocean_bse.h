/*
 * ocean_bse.h -- C ABI of the MI355X (gfx950) core-level BSE solver library.
 *
 * The library evaluates the action of the Bethe-Salpeter Hamiltonian of a
 * core-level excitation on exciton vectors, runs the Haydock (Lanczos) recursion
 * with it, and turns the recursion coefficients into a spectrum, as stated in
 * Gilmore et al., "Efficient implementation of core-excitation Bethe-Salpeter
 * equation calculations":
 *
 *   sigma(w) ~ -(1/pi) Im <0| O+ G(w) O |0>,  G(w) = [w - H_BSE]^-1      (section 2, eq. loss.fcn)
 *   H_BSE = H_e - H_h - V_D + V_X                                         (section 2, eq. H_BSE)
 *   the exciton vector psi_{alpha,n,k}                                    (section 3.2)
 *   W0 (long-range direct) applied as in Algorithm 1                      (section 3.2.1)
 *   short-range direct + exchange through a local basis                   (section 3.2.2, eq. local_basis)
 *   the Haydock iteration psi^{i+1} = H psi^i                             (section 3.2, eq. haydock1)
 *
 * Conventions used by every entry point
 * -------------------------------------
 *  - Complex numbers are pairs of doubles (re, im), i.e. C99 double _Complex /
 *    numpy complex128 / torch.complex128 memory layout.
 *  - Energies in Hartree, lengths in bohr.
 *  - Grids: a cell of any shape given by its lattice vectors a_1, a_2, a_3 (the rows of
 *    ocean_bse_desc.cell, bohr) and the reciprocal vectors b_d with a_i . b_j = 2 pi delta_ij;
 *    k grid k = sum_d ((i_d + s_d) / nk_d) b_d, i_d = 0 .. nk_d - 1 (s_d = 0 is the
 *    Gamma-centred grid; an offset s_d needs no input, see ocean_bse_desc.cell); real-space
 *    points x = sum_d (j_d / nx_d) a_d; lattice vectors of the Born-von-Karman supercell
 *    R = sum_d r_d a_d, r_d = 0 .. nk_d - 1.  Flat grid indices are row-major with the last
 *    axis fastest.
 *  - An exciton vector is stored [k][n][c]: k-point slowest, core index c fastest,
 *    Nk*Nb*Nc complex numbers.  n_vec vectors are stored one after another.
 *  - Core index for an L2,3 edge: c = (m_c + 1) * 2 + sigma (sigma = 0 spin up);
 *    for a K edge: c = sigma.  Local channel index mu = m + 2 (d channel, m = -2..2).
 *  - Return codes: 0 = OK, > 0 informational, < 0 error.  After an error,
 *    ocean_last_error() returns a message for the calling thread.  No entry
 *    point aborts or throws across the ABI.
 *  - Device pointers are HIP device allocations on the current device.  All
 *    device work of a handle is enqueued on the handle's stream; entry points
 *    that return host results synchronise that stream first.
 *  - Handles are not thread-safe: calls on one handle must not overlap.
 */
#ifndef OCEAN_BSE_H
#define OCEAN_BSE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ocean_bse_s* ocean_bse_t;

enum {
    OCEAN_OK = 0,
    OCEAN_INFO_INVARIANT_SUBSPACE = 1, /* Haydock stopped early: b_{i+1} ~ 0 */
    OCEAN_ERR_INVALID_ARG = -1,
    OCEAN_ERR_OUT_OF_MEMORY = -2,
    OCEAN_ERR_DEVICE = -3,
    OCEAN_ERR_UNSUPPORTED = -4
};

/* Storage / arithmetic precision of the two band-projection contractions
 * (the band-to-real-space and real-space-to-band steps of Algorithm 1).  Everything else -- the diagonal, core and local
 * terms, the Lanczos inner products, norms, coefficients and the continued
 * fraction -- is FP64 in every mode. */
enum {
    OCEAN_PREC_FP64 = 0,       /* u_nk in FP64, FP64 MFMA */
    OCEAN_PREC_FP32 = 1,       /* u_nk stored FP32, FP32 MFMA, FP32 accumulation */
    OCEAN_PREC_SPLIT_BF16 = 2, /* u_nk stored as bf16 hi + residual planes (8 B per complex), the vector split
                                  into hi + residual when staged; 3 bf16 MFMA products, FP32 accumulation */
    OCEAN_PREC_BF16 = 3        /* u_nk stored as one bf16 plane (4 B per complex), the vector split into hi +
                                  residual; 2 bf16 MFMA products, FP32 accumulation.  The error is set by
                                  the bf16 rounding of u_nk (relative 2^-9 per element). */
};

/* ocean_bse_desc.flags */
#define OCEAN_FLAG_BORROW_DEVICE_U 0x1u  /* desc.u is a device pointer: in FP64 mode the handle uses it in
                                            place (it must outlive the handle); in the FP32 and bf16
                                            modes it is only read during ocean_bse_create */
#define OCEAN_FLAG_CHECK_INPUTS    0x2u  /* scan inputs for NaN/Inf and check Hermiticity of the small matrices */

/* ocean_haydock flags */
#define OCEAN_HAYDOCK_REORTH 0x1u  /* full re-orthogonalisation (two classical Gram-Schmidt passes) each step */

/* ocean_spectrum terminators */
enum { OCEAN_TERM_NONE = 0, OCEAN_TERM_SQRT = 1 };

/* Description of one crystal / core site (the inputs of the BSE stage, section 2
 * and section 3.2).  All host arrays are copied by ocean_bse_create; the caller may
 * free them when it returns. */
typedef struct {
    int nk[3];            /* k grid (and Born-von-Karman supercell) n1 x n2 x n3, each >= 1 */
    int nx[3];            /* real-space grid of one cell g1 x g2 x g3, each >= 1 */
    int n_bands;          /* Nb >= 1 conduction bands per k */
    int n_core;           /* Nc core states, 1..12 (2: 1s with spin, 6: 2p with spin, 12: 2p with
                             the electron spin carried separately) */
    int n_local;          /* Nmu >= 0 local functions (<= 64; n_core * n_local <= 768); 0 disables the
                             short-range term */
    double cell[3][3];    /* rows: lattice vectors a1, a2, a3 of the cell, bohr, any shape with
                             nonzero volume.  Grid point j of the cell is x = sum_d (j_d / g_d) a_d,
                             lattice vector r of the supercell is R = sum_d r_d a_d.  The minimum
                             image of x + R - tau in the Born-von-Karman supercell (rows n_d a_d) is
                             taken over the 27 translations around its wrapped fractional
                             coordinates: exact for a reduced (not strongly skewed) basis.
                             A k grid offset by a fraction of a step needs no input: the offset
                             cancels in W0 (only k - k' enters), so u_nk and E_nk at the offset
                             points are all that changes. */
    double tau[3];        /* absorbing-site position, bohr */
    const double* energies;   /* [Nk][Nb] real, Ha: H_e eigenvalues E_nk (section 2) of the band
                                 window.  Absorption passes the unoccupied bands; emission
                                 (XES) passes the occupied bands, energies below the Fermi
                                 level, with the same operator (the lines then sit at
                                 E_nk - E_c, E_c = 0). */
    const double* u;          /* [Nk][Nx][Nb] complex: periodic Bloch parts u_nk(x), columns
                                 orthonormal per k (sum_x |u|^2 = 1).  Host pointer, or a
                                 device pointer with OCEAN_FLAG_BORROW_DEVICE_U. */
    int n_wr;                 /* number of radial table points, >= 2 */
    const double* w_r;        /* [n_wr] radii, bohr: uniform, w_r[0] = 0, ascending */
    const double* w_val;      /* [n_wr] W0(r), Ha (section 3.2.1); linear interpolation
                                 between nodes and W(r_max) r_max / r beyond the last node */
    const double* local_proj; /* [Nk][Nb][Nmu] complex A^{mu}_{nk} (eq. local_basis) or NULL */
    const double* local_mat;  /* [(Nc Nmu)^2] complex, row-major over pairs (c, mu) -> c*Nmu+mu:
                                 the short-range direct + exchange matrix (section 3.2.2), Hermitian, or NULL */
    const double* core_mat;   /* [Nc^2] complex, row-major: -(eps_c + chi) acting on the core index
                                 (the -H_h term of eq. H_BSE), Hermitian, or NULL */
    int precision;            /* OCEAN_PREC_* */
    unsigned flags;           /* OCEAN_FLAG_* */
} ocean_bse_desc;

/* Create a solver handle: uploads and converts u_nk, builds the W(x, R) table of
 * the Born-von-Karman supercell (minimum image, section 3.2.1) and the phase
 * tables of Algorithm 1.  stream: a hipStream_t to enqueue on, or NULL for a
 * stream owned by the handle.  On success *out is a new handle.
 * Errors: INVALID_ARG (bad sizes, NULL required arrays, NaN with CHECK_INPUTS,
 * non-uniform radial grid), OUT_OF_MEMORY (device allocation failed or would
 * exceed OCEAN_MAX_DEVICE_BYTES if that environment variable is set), DEVICE. */
int ocean_bse_create(const ocean_bse_desc* desc, void* stream, ocean_bse_t* out);

/* Release every device allocation of the handle (borrowed u is not freed). */
void ocean_bse_destroy(ocean_bse_t h);

/* Dimension Nk*Nb*Nc of one exciton vector (complex elements), or < 0 on error. */
long long ocean_bse_dim(ocean_bse_t h);

/* y = H_BSE x for n_vec >= 1 vectors (section 3.2: the sum of the diagonal,
 * core-matrix, long-range W0 of Algorithm 1, and short-range local pieces).
 * x_dev, y_dev: device arrays of n_vec * dim complex numbers, layout [v][k][n][c];
 * they must not overlap.  Enqueued on the handle's stream; returns without
 * synchronising.  Errors: INVALID_ARG (NULL pointers, n_vec < 1), OUT_OF_MEMORY
 * (workspace growth), DEVICE (launch failure). */
int ocean_bse_apply(ocean_bse_t h, const double* x_dev, double* y_dev, int n_vec);

/* Haydock recursion (section 3.2, eq. haydock1, as the three-term Lanczos
 * recursion) for n_vec independent starting vectors psi0_dev ([v][k][n][c]
 * complex, device, not modified):
 *   v_0 = psi0/|psi0|, b_0 = 0;  w = H v_i;  a_i = Re<v_i|w>;
 *   w -= a_i v_i + b_i v_{i-1};  b_{i+1} = |w|;  v_{i+1} = w / b_{i+1}.
 * Host outputs: a[v*n_steps + i] = a_i, b[v*n_steps + i] = b_{i+1} for i < n_steps,
 * norm2[v] = |psi0_v|^2, steps_done[v] = completed steps.  A vector stops early
 * (its remaining a, b entries are 0) when b_{i+1} <= 1e-14 max(|a_0..a_i|, b_1..b_i);
 * the call then returns OCEAN_INFO_INVARIANT_SUBSPACE.  All inner products and
 * norms are FP64 with a fixed reduction order (bitwise reproducible run to run).
 * flags: OCEAN_HAYDOCK_REORTH.  Synchronises the handle's stream.
 * Errors: INVALID_ARG (NULL pointers, n_vec < 1, n_steps < 1, psi0 = 0),
 * OUT_OF_MEMORY, DEVICE. */
int ocean_haydock(ocean_bse_t h, const double* psi0_dev, int n_vec, int n_steps, unsigned flags,
                  double* a, double* b, double* norm2, int* steps_done);

/* Checkpoint and resume of the recursion.  Each Haydock step (section 3.2, eq. haydock1)
 * needs only v_i, v_{i-1} and b_i besides H; the coefficients already produced are the
 * caller's.  So the state of a recursion is the two vectors plus, per vector,
 * OCEAN_HAYDOCK_STATE_LEN doubles: {b_i, the running breakdown scale max(|a|, b), |psi0|^2,
 * a_{i-1}, stopped (0 or 1), steps of the last call}.
 *
 * ocean_haydock_export copies the state the last ocean_haydock / ocean_haydock_batch /
 * ocean_haydock_continue call on this handle ended in: v_dev and vprev_dev are device
 * buffers of n_vec * dim complex (caller-owned), state is host [n_vec][6].  n_vec must be
 * that call's.  Synchronises the handle's stream.  Errors: INVALID_ARG (NULL, no such
 * run), DEVICE.
 *
 * ocean_haydock_continue runs n_steps more steps from such a state, on this handle or on
 * another handle of the same system: a[v*n_steps + j], b[v*n_steps + j] are the next
 * coefficients (a_{i+j}, b_{i+j+1}), steps_done[v] the steps completed in this call.  The
 * coefficients of a run split this way equal those of one uninterrupted run bit for bit.
 * Without re-orthogonalisation only (it would need every earlier vector).  Returns
 * OCEAN_INFO_INVARIANT_SUBSPACE as ocean_haydock does (a vector that had already stopped
 * completes 0 steps).  Errors: INVALID_ARG (NULL, n_vec or n_steps < 1, a state that no
 * export wrote), UNSUPPORTED (OCEAN_HAYDOCK_REORTH), OUT_OF_MEMORY, DEVICE. */
#define OCEAN_HAYDOCK_STATE_LEN 6
int ocean_haydock_export(ocean_bse_t h, int n_vec, double* v_dev, double* vprev_dev, double* state);
int ocean_haydock_continue(ocean_bse_t h, const double* v_dev, const double* vprev_dev, const double* state,
                           int n_vec, int n_steps, unsigned flags, double* a, double* b, int* steps_done);

/* Batched Haydock recursion for n_sys independent systems (sites, edges,
 * polarisations: section 4.3 keeps the wavefunctions resident and amortises them over
 * many spectra; section 4.5 runs hundreds of site-edge calculations).  System s uses
 * handle hs[s] (distinct handles with distinct streams, one device), starting vectors
 * psi0[s] (device, n_vec[s] vectors as in ocean_haydock).  Up to 8 steps of every system
 * (OCEAN_BATCH_CHAIN in the environment sets the count) are captured into a single HIP graph,
 * each system an independent branch whose steps follow one another with no join between
 * systems, and the graph is replayed until n_steps steps are done.  Host outputs are concatenated over systems in order: vector j of the batch
 * (systems in order, their vectors in order) has a[j*n_steps + i], b[j*n_steps + i],
 * norm2[j], steps_done[j].  Each system's numbers are bitwise those of ocean_haydock on
 * the same handle.  Returns OCEAN_INFO_INVARIANT_SUBSPACE if any vector stopped early.
 * Errors: INVALID_ARG (NULL, shared handle or stream, mixed devices, zero psi0),
 * OUT_OF_MEMORY, DEVICE. */
int ocean_haydock_batch(const ocean_bse_t* hs, int n_sys, const double* const* psi0,
                        const int* n_vec, int n_steps, unsigned flags, double* a, double* b,
                        double* norm2, int* steps_done);

/* Tile autotuner (not in the paper: the kernels of Algorithm 1, section 3.2.1, have tile
 * shapes that depend on the system): times the candidate tile shapes of the projection,
 * back-projection and k-grid transform kernels on this handle's shape with n_vec vectors (mean of the
 * tuned kernel's own HIP-event time over reps applies per candidate, after one untimed
 * apply; reps < 1 means 5) and keeps the fastest.  If the environment variable
 * OCEAN_AUTOTUNE_CACHE names a file, a cached choice for the same shape and the same version
 * of the kernels is reused when every knob is one the tuner itself could have picked (any
 * other line is ignored and the shape is tuned again), and new choices are appended.  Results
 * do not change numerics beyond summation order of the split-K partials.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
int ocean_bse_autotune(ocean_bse_t h, int n_vec, int reps);

/* Current tile choices: forward rows per wave / 16, back-projection grid target, lines
 * per k-grid transform block, row tiles per block of the FP64/FP32 forward projection that
 * keeps psi[k] of every band resident in LDS (0: the band-chunked forward; the resident form
 * applies only where psi[k] of a pass fits in 64 KiB), and the most waves (16 bands each) per
 * back-projection block (the 16-band groups are dealt evenly over the fewest blocks that
 * respect it: 96 bands at 4 make two blocks of 3 waves).  Any pointer may be NULL.
 * Environment overrides at create: OCEAN_BWD_BLOCKS, OCEAN_FWD_TILES, OCEAN_BWD_WAVES (1..8).
 * Errors: INVALID_ARG. */
int ocean_bse_get_tuning(ocean_bse_t h, int* fwd_ms, int* bwd_blocks, int* fft_lines, int* fwd_tiles,
                         int* bwd_waves);

/* Spectra from Haydock coefficients (section 2, eq. loss.fcn with
 * G = [w - H]^-1 as a continued fraction), evaluated on the GPU in FP64:
 *   sigma(w) = -(1/pi) norm2 Im g(w + i gamma),
 *   g(z) = 1/(z - a_0 - b_1^2/(z - a_1 - ... - b_{N-1}^2/(z - a_{N-1} - b_N^2 t(z)))).
 * Host inputs: a, b [n_spec][n_steps] as written by ocean_haydock, n_used[s]
 * (levels to use, <= n_steps; NULL = n_steps), norm2 [n_spec], omega [n_omega] (Ha).
 * gamma (Ha, > 0) is the Lorentzian half width.  terminator: OCEAN_TERM_NONE (t = 0)
 * or OCEAN_TERM_SQRT (the Green's function of a semi-infinite chain with constant
 * coefficients a_inf, b_inf: t = [(z - a_inf) - sqrt((z - a_inf)^2 - 4 b_inf^2)] / (2 b_inf^2),
 * the root with Im t <= 0).  a_inf, b_inf: host [n_spec] (both given, finite, b_inf > 0), or
 * both NULL for the means of the last 16 used a_i and b_{i+1}; ignored with
 * OCEAN_TERM_NONE.  The learned terminator of the recursion's tail is the composition
 * ocean_mlp_predict (the coefficients extended to 256 levels) then OCEAN_TERM_SQRT on the
 * extended chain.  Host output sigma [n_spec][n_omega].  Synchronous; uses its own stream.
 * Errors: INVALID_ARG (also a_inf without b_inf or the reverse), OUT_OF_MEMORY, DEVICE. */
int ocean_spectrum(const double* a, const double* b, const int* n_used, const double* norm2,
                   int n_spec, int n_steps, int terminator, const double* a_inf, const double* b_inf,
                   const double* omega, int n_omega, double gamma, double* sigma);

/* ---- Learned continued-fraction terminator ------------------------------------------
 * Not part of the paper: a small network that extends the Haydock coefficients of
 * section 3.2 from the first 32 pairs to 256, so that the continued fraction of
 * eq. loss.fcn needs 32 H*v instead of hundreds.  Network 64 -> 256 -> 256 -> 256 -> 448,
 * ReLU, mean-squared error (optionally weighted per output position), Adam (beta1 0.9, beta2
 * 0.999, eps 1e-8).  Parameters are
 * FP32 masters packed [W1, b1, W2, b2, W3, b3, W4, b4] with W stored [in][out]
 * (ocean_mlp_param_count() floats).  The GEMMs run on the matrix cores: bf16 inputs
 * with FP32 accumulation (OCEAN_MLP_BF16), or FP32 inputs (OCEAN_MLP_FP32).
 * Encoding per sequence: c = mean(a_16..a_31), s = mean(b_17..b_32); input
 * [(a_n - c)/s, b_{n+1}/s] for n < 32; output [(a_n - c)/s, log(b_{n+1}/s)] for
 * 32 <= n < 256.  A handle owns its own stream; calls synchronise it before returning
 * host data.  Not thread-safe. */
typedef struct ocean_mlp_s* ocean_mlp_t;
enum { OCEAN_MLP_BF16 = 0, OCEAN_MLP_FP32 = 1 };

/* Number of packed parameters (263360). */
int ocean_mlp_param_count(void);
/* New network with zero parameters.  Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
int ocean_mlp_create(int precision, ocean_mlp_t* out);
void ocean_mlp_destroy(ocean_mlp_t h);
/* Copy parameters in (host, resets the Adam moments and step count) or out (host). */
int ocean_mlp_set_params(ocean_mlp_t h, const float* params);
int ocean_mlp_get_params(ocean_mlp_t h, float* params);
/* Weight of each output position in the mean-squared error of ocean_mlp_loss_grad and
 * ocean_mlp_train_step: loss = sum_{s, j} w_j (y_sj - t_sj)^2 / (batch * 448).  w is host [448]
 * (finite, >= 0), copied; NULL restores unit weights.  Errors: INVALID_ARG, OUT_OF_MEMORY,
 * DEVICE. */
int ocean_mlp_set_loss_weights(ocean_mlp_t h, const float* w);
/* Checkpoint: write the parameters, the Adam moments and step count to the file at path
 * (binary, little-endian: the 8 bytes "OCEANMLP", int32 version 1, int32 precision,
 * int32 Adam step, int32 parameter count, then three float32 arrays of that count:
 * parameters, first moments, second moments), or restore them from such a file so that
 * training resumes exactly where it stopped.  The precision stored must match the
 * handle's.  Synchronous.  Errors: INVALID_ARG (NULL argument, unreadable or unwritable
 * file, wrong format, count or precision), DEVICE. */
int ocean_mlp_save(ocean_mlp_t h, const char* path);
int ocean_mlp_load(ocean_mlp_t h, const char* path);
/* Features x [n_seq][64] and, when t_dev is not NULL, targets t [n_seq][448] (device,
 * FP32) from coefficient sequences a, b [n_seq][stride] (device, FP64, b[j] = b_{j+1});
 * stride >= 32, or >= 256 with targets.  Synchronous.  Errors: INVALID_ARG, DEVICE. */
int ocean_mlp_encode(const double* a_dev, const double* b_dev, int n_seq, int stride, float* x_dev,
                     float* t_dev);
/* y [batch][448] = network(x [batch][64]); device arrays.  Synchronous. */
int ocean_mlp_forward(ocean_mlp_t h, const float* x_dev, int batch, float* y_dev);
/* Loss and gradient of the (weighted, see ocean_mlp_set_loss_weights) mean-squared error over
 * the batch; loss (host) and grad (host, packed like the parameters) may each be NULL.
 * Synchronous. */
int ocean_mlp_loss_grad(ocean_mlp_t h, const float* x_dev, const float* t_dev, int batch,
                        double* loss, float* grad);
/* One Adam step on the batch (forward, backward, update) with learning rate lr.  Returns
 * the batch loss in *loss if not NULL (then synchronous; otherwise asynchronous). */
int ocean_mlp_train_step(ocean_mlp_t h, const float* x_dev, const float* t_dev, int batch, float lr,
                         double* loss);
/* Extended coefficients for n_seq sequences (host a, b [n_seq][stride], stride >= 32):
 * a_ext, b_ext [n_seq][256] hold the given first 32 pairs followed by the 224 predicted
 * ones; valid[s] = 0 flags a sequence whose prediction is not finite or has b <= 0 (the
 * caller then falls back to full-depth Haydock).  Synchronous. */
int ocean_mlp_predict(ocean_mlp_t h, const double* a, const double* b, int n_seq, int stride,
                      double* a_ext, double* b_ext, int* valid);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops
 * or harnesses that forbid hipMalloc): ocean_mlp_predict on device buffers, allocating nothing.
 * Inputs a_dev, b_dev [n_seq][stride] (device, FP64, b[j] = b_{j+1}, stride >= 32); outputs
 * a_ext_dev, b_ext_dev [n_seq][256] (device, FP64) and valid_dev [n_seq] (device, int), with the
 * meaning of ocean_mlp_predict's (results equal that call's bit for bit).  The encoding
 * constants and the activations of every layer live in one fixed array of device memory of
 * about 21 MB (OCEAN_MLP_NOALLOC_MAX_SEQ sequences at most), which each device that the library
 * runs on holds until the process ends; its address is resolved once per device by
 * ocean_mlp_create.  Every call on one device shares that array and every element a call reads
 * is written by the same call first, so nothing carries over between calls, but calls that
 * overlap on one device (other streams, other threads, other handles) race: the caller must
 * serialise them.  Enqueued on `stream` (a hipStream_t on the handle's device, or NULL for the
 * default stream); returns without synchronising.  The parameters are read on that stream, so
 * work still pending on the handle's own stream (an asynchronous ocean_mlp_train_step) must
 * have finished first.  Calls no hipMalloc, hipFree or other allocating routine.
 * Errors: INVALID_ARG (NULL, n_seq < 1 or > OCEAN_MLP_NOALLOC_MAX_SEQ, stride < 32), DEVICE
 * (launch failure). */
#define OCEAN_MLP_NOALLOC_MAX_SEQ 4096
int ocean_mlp_predict_noalloc(ocean_mlp_t h, const double* a_dev, const double* b_dev, int n_seq, int stride,
                              double* a_ext_dev, double* b_ext_dev, int* valid_dev, void* stream);

/* Host helper: the L2,3-edge (2p core, d channel) matrices for ocean_bse_desc
 * from the spin-orbit parameter zeta and the Slater integrals F2 (screened
 * direct) and G1, G3 (bare exchange), all in Ha (section 2: H_h, V_D, V_X;
 * section 3.2.2: multipole expansion with selection rules).
 * core_mat [6*6] complex = -chi with chi = zeta l.s; local_mat [30*30] complex =
 * -(D x I_spin) + (X x J_spin) with D = F2 c^2(2m';2m) c^2(1mc';1mc) and
 * X = sum_{k=1,3} G^k c^k(2m';1mc') c^k(2m;1mc), c^k the Gaunt coefficients.
 * Either output may be NULL.  Errors: INVALID_ARG. */
int ocean_multiplet_matrices(double zeta, double F2, double G1, double G3,
                             double* core_mat, double* local_mat);

/* Host helper: the same matrices on the full electron x hole spin space (section 3.2.2:
 * the electron and hole spins carried separately), for n_core = 12 with core index
 * ((m_c + 1) * 2 + sigma_h) * 2 + sigma_e.  core_mat [12*12] complex = -chi on (m_c, sigma_h),
 * the identity on sigma_e; local_mat [60*60] complex on pairs (core index, m) ->
 * core index * 5 + (m + 2):
 *   -D delta(sigma_h', sigma_h) delta(sigma_e', sigma_e) + X delta(sigma_h', sigma_e') delta(sigma_h, sigma_e),
 * with D and X as above: the direct term keeps both spins, the exchange term annihilates a
 * pair of equal spins and creates another.  On the pairs with sigma_e = sigma_h this is the
 * restricted matrix.  Either output may be NULL.  Errors: INVALID_ARG. */
int ocean_multiplet_matrices_spin(double zeta, double F2, double G1, double G3,
                                  double* core_mat, double* local_mat);

/* Host helper: the short-range matrix of a general local basis (section 3.2.2: radial
 * projectors for each l, the multipole expansion with its selection rules).  n_ch channels,
 * channel i with angular momentum l[i] in 0..3 (several channels may share an l: the radial
 * functions); local index mu = (channel, m = -l..l) in that order, N_mu = sum (2 l + 1) <= 64.
 *   f2 [n_ch][n_ch]     screened direct radial integrals F^2 (F^0 is the long-range W0);
 *   gk [5][n_ch][n_ch]  bare exchange radial integrals G^k, k = 0..4 (only the k that the
 *                       Gaunt selection rules allow for a 2p core contribute).
 *   D[(m_c', i', m'), (m_c, i, m)] = F2[i'][i] c^2(l_i' m'; l_i m) c^2(1 m_c'; 1 m_c),
 *   X[(m_c', i', m'), (m_c, i, m)] = sum_k G^k[i'][i] c^k(l_i' m'; 1 m_c') c^k(l_i m; 1 m_c),
 * assembled with the spin structure of ocean_multiplet_matrices (full_spin = 0: core index
 * (m_c, sigma), N_c = 6) or of ocean_multiplet_matrices_spin (full_spin = 1, N_c = 12).
 * local_mat: [(N_c N_mu)^2] complex, pair index core index * N_mu + mu.  With one d channel,
 * f2 = F2 and gk = {G1, G3 at k = 1, 3} this is ocean_multiplet_matrices' matrix.
 * Errors: INVALID_ARG (NULL, l out of range, non-finite), UNSUPPORTED (N_mu > 64). */
int ocean_local_matrix_channels(int n_ch, const int* l, const double* f2, const double* gk, int full_spin,
                                double* local_mat);

/* Host helper: dipole amplitudes (section 2, eq. loss.fcn, O = e.r) of a general local
 * basis (section 3.2.2, eq. local_basis), d[mu][mc+1] = radial[i] <Y_{l_i m}| e.r^ |Y_1mc>
 * for mu = (channel i, m); only s and d channels couple to a 2p core.  d is [N_mu][3]
 * complex.  Errors: INVALID_ARG. */
int ocean_dipole_amplitudes_channels(int n_ch, const int* l, const double* radial, const double* e, double* d);

/* Host helper: dipole amplitudes d[m+2][mc+1] = <Y_2m| e.r^ |Y_1mc> (radial
 * integral 1) for a polarisation e[3] (section 2: O = e.r for XAS).  d is [5][3]
 * complex.  Errors: INVALID_ARG. */
int ocean_dipole_amplitudes(const double* e, double* d);

/* Initial vectors O|0> for an L2,3 edge on the device (section 2, eq. loss.fcn;
 * eq. local_basis): psi0[p][k][n][(mc, s)] = sum_m conj(A[k][n][m]) d_p[m][mc] for
 * n_pol polarisations pol[p][3], the same for both spins (Nc = 6).  With the electron spin
 * carried separately (Nc = 12, index ((mc, s_h), s_e)) the amplitude sits on s_e = s_h
 * and the other pairs are zero.  Needs Nc = 6 or 12 and Nmu = 5.  psi0_dev: device, n_pol * dim complex.  Enqueued on the handle's
 * stream.  Errors: INVALID_ARG, UNSUPPORTED (other edge shapes), DEVICE. */
int ocean_dipole_psi0(ocean_bse_t h, const double* pol, int n_pol, double* psi0_dev);

/* The same for a general local basis (section 3.2.2): channels l[n_ch] with radial dipole integrals
 * radial[n_ch] (ocean_dipole_amplitudes_channels), spanning exactly the handle's n_local
 * functions; n_core 6 or 12 (spin layout as in ocean_dipole_psi0).  Errors: INVALID_ARG,
 * UNSUPPORTED (other shapes), DEVICE. */
int ocean_dipole_psi0_channels(ocean_bse_t h, int n_ch, const int* l, const double* radial, const double* pol,
                               int n_pol, double* psi0_dev);

/* Host helper: amplitudes of the non-resonant scattering operator e^{iq.r} (section 2,
 * eq. loss.fcn: the operator named there for NRIXS) on a general local basis.  With the
 * plane-wave expansion e^{iq.r} = 4 pi sum_{LM} i^L j_L(qr) conj(Y_LM(q^)) Y_LM(r^),
 *   d[mu][mc+1] = sum_L radial[i][L] i^L sqrt(4 pi (2L+1)) conj(Y_{L,m-mc}(q^)) c^L(l_i m; 1 mc)
 * for mu = (channel i, m), where radial[i][L] = int R_i(r) j_L(|q| r) R_2p(r) r^2 dr is the
 * caller's (row-major [n_ch][n_L], 1 <= n_L <= 16; terms with L > l_i + 1 vanish).  q[3] is
 * the momentum transfer (nonzero; only its direction enters here).  d is [N_mu][3] complex.
 * Errors: INVALID_ARG (NULL, l out of 0..3, n_L out of range, non-finite, q = 0). */
int ocean_nrixs_amplitudes_channels(int n_ch, const int* l, int n_L, const double* radial, const double* q,
                                    double* d);

/* Host helper: XAS amplitudes with the first term beyond the dipole (section 2, eq. loss.fcn:
 * O = e.r + (i/2)(e.r)(q.r)),
 *   d[mu][mc+1] = radial1[i] <Y_lm| e.r^ |Y_1mc> + (i/2) radial2[i] <Y_lm| (e.r^)(q.r^) |Y_1mc>,
 * radial1[i] and radial2[i] the channel's integrals of r and r^2 against the 2p function,
 * e[3] a real polarisation and q[3] the photon wave vector (any length; q = 0 gives the
 * dipole amplitudes).  d is [N_mu][3] complex.  Errors: INVALID_ARG. */
int ocean_quadrupole_amplitudes_channels(int n_ch, const int* l, const double* radial1, const double* radial2,
                                         const double* e, const double* q, double* d);

/* Initial vectors O|0> on the device for any transition operator given by its local
 * amplitudes (section 2, eq. loss.fcn; eq. local_basis): d is host [n_pol][N_mu][3] complex
 * (from the helpers above, or the caller's own), and psi0[p][k][n][core] =
 * sum_mu conj(A[k][n][mu]) d_p[mu][mc] with the spin layout of ocean_dipole_psi0.  Needs
 * n_core 6 or 12.  psi0_dev: device, n_pol * dim complex.  Errors: INVALID_ARG (NULL,
 * non-finite), UNSUPPORTED (other core shapes), DEVICE. */
int ocean_psi0_amplitudes(ocean_bse_t h, const double* d, int n_pol, double* psi0_dev);

/* Per-kernel timing.  While enabled, every launch of the handle is bracketed by
 * HIP events on the handle's stream and its duration is accumulated per kernel
 * name.  ocean_bse_kernel_times copies up to max_entries (name, total ms, launch
 * count) triples; names are static strings owned by the library.  Returns the
 * number of entries, or < 0 on error.  Enabling or resetting clears the totals. */
int ocean_bse_set_profiling(ocean_bse_t h, int enable);
int ocean_bse_kernel_times(ocean_bse_t h, const char** names, double* total_ms,
                           long long* counts, int max_entries);

/* Device bytes currently held by the handle (inputs, converted copies, tables,
 * workspace), or < 0 on error. */
long long ocean_bse_device_bytes(ocean_bse_t h);

/* ---- Screening response (section 3.3) ---------------------------------------------------
 * Static RPA response chi0 on the real-space grid around the core site (eq. chi_rpa at
 * omega = 0, with the Green's function of eq. greens.fcn):
 *   G_j(r, r') = sum_s psi_s(r) psi_s*(r') / (mu + i t_j - eps_s),
 *   chi0(r, r') = sum_j (w_j / pi) Re[G_j(r, r') G_j(r', r)],
 * i.e. the frequency integral along the imaginary axis through the chemical potential mu,
 * folded onto t >= 0 (the integrand at -t is the conjugate of the one at t), with nodes t_j
 * and weights w_j chosen by the caller.  One spin channel.
 *   psi_dev   device, [n_points][n_states] complex (row-major, states fastest): the Bloch
 *             functions of every state summed over (all bands and k) on the grid points.
 *   eps       host, [n_states] energies (Ha); mu (Ha); t, w host [n_t], t_j >= 0.
 *   chi0_dev  device, [n_points][n_points] real (row-major), overwritten.  Real and symmetric.
 * With A_j = Psi diag(Re d_j) Psi^H and B_j = Psi diag(Im d_j) Psi^H (d_j(s) = 1/(mu + i t_j - eps_s)),
 * Re[G_j(r, r') G_j(r', r)] = |A_j(r, r')|^2 - |B_j(r, r')|^2: one FP64 matrix-core kernel forms A_j and
 * B_j tile by tile (upper-triangle tile pairs) and accumulates that expression; G_j is never stored.
 * Node partials are added in node order, so results are bitwise reproducible.
 * stream: hipStream_t or NULL for the default stream; the call returns after the work has
 * finished.  Uses n_t * n_points^2 + n_states + 2 n_t doubles of device scratch (the node
 * partials), allocated on the current device at the first call that needs that much and kept
 * between calls until ocean_screening_release; calls are serialised by the library (they share
 * the scratch).
 * Errors: INVALID_ARG (NULL, sizes < 1, non-finite input, negative node), OUT_OF_MEMORY,
 * DEVICE. */
int ocean_screening_chi0(const double* psi_dev, const double* eps, int n_points, int n_states,
                         double mu, const double* t, const double* w, int n_t, double* chi0_dev,
                         void* stream);

/* Free the device scratch that ocean_screening_chi0 keeps between calls, on every device that
 * holds one.  The next build allocates it again.  Errors: DEVICE. */
int ocean_screening_release(void);

/* Measured ceilings of the current device, for the roofline of the projections of
 * Algorithm 1 (section 3.2.1), which issue FP64 matrix-core instructions, FP64 multiply-adds
 * and an HBM stream:
 *   mfma_f64_tflops  16x16x4 FP64 MFMAs, four independent accumulators per wave, four waves
 *                    per SIMD (TFLOP/s, 2 flops per multiply-add);
 *   fma_f64_tflops   wave-wide FP64 multiply-adds, eight independent chains per lane;
 *   copy_gbs         a copy of copy_bytes (>= 1 MiB), one 16-byte element per thread, bytes
 *                    read plus bytes written per second (GB/s);
 *   read_gbs         a read of the same copy_bytes, 1024 consecutive 16-byte elements per
 *                    block (GB/s).
 * Each figure is the fastest of three timed launches after an untimed one.  Allocates and frees 2 copy_bytes
 * of device memory plus small result buffers; synchronous, on a private stream.
 * Errors: INVALID_ARG (copy_bytes < 1 MiB, NULL output), OUT_OF_MEMORY, DEVICE. */
int ocean_device_ceilings(long long copy_bytes, double* mfma_f64_tflops, double* fma_f64_tflops,
                          double* copy_gbs, double* read_gbs);

/* Message describing the last error on the calling thread ("" if none). */
const char* ocean_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* OCEAN_BSE_H */
