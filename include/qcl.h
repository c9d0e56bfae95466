/*
 * qcl.h -- C ABI of the MI355X (gfx950) propagator for the
 * momentum-jump-free quantum-classical Liouville (QCL) trajectory ensemble
 * (K. Ando, "GPU implementation of mixed quantum-classical Liouville
 * molecular dynamics without momentum jump").
 *
 * The method (Sec. II.A, Eq. 1) propagates the partially Wigner-transformed
 * density matrix rho_ab:W(R,P) with a fixed number of independent walkers
 * (Sec. II.B: no trajectory spawning).  A walker carries one element (a,b)
 * of the adiabatic basis, classical coordinates q and momenta p, a real
 * weight w and a phase Phi; its contribution to rho_ab is w exp(-i Phi).
 * Per step it makes a Monte Carlo move between elements with a weight
 * update (the -(P/M) sum_g (d rho - rho d) term; p is never changed),
 * moves (q,p) by velocity Verlet on the mean force (F_a + F_b)/2 (last two
 * terms of Eq. 1) and accumulates Phi from w_ab = (E_a - E_b)/hbar (first
 * term of Eq. 1).  Ensemble averages are reduced in a fixed order
 * (Sec. II.B: deterministic reduction rather than atomics).
 *
 * Model family: linear-vibronic harmonic Hamiltonians (Sec. II.C models)
 *     H = sum_j p_j^2/(2 m_j) + sum_j m_j w_j^2 q_j^2/2 + V0 + sum_j q_j K_j
 * with real symmetric N x N matrices V0 and K_j.
 *
 * General conventions
 *   - Every call returns a qcl_status; nothing throws across the ABI.  On
 *     failure qcl_last_error() returns a thread-local message.
 *   - Arguments are validated on the host before any launch; an invalid
 *     call launches nothing and changes nothing.
 *   - "device" pointers are HIP device allocations owned by the caller;
 *     "host" pointers are read during the call only.
 *   - Device work is enqueued on the given stream (a hipStream_t passed as
 *     void*, NULL = the default stream) and is asynchronous: results are
 *     valid once the stream has reached the point of the call.
 *   - Nothing in qcl_sample_initial, qcl_propagate or
 *     qcl_reduce_observables allocates memory.
 *   - Every device pointer (ensemble arrays, partials, out, workspaces) must
 *     be 256-byte aligned (INVALID_ARG otherwise); qcl_ensemble_bind and
 *     allocations of the HIP and torch allocators are.
 *   - A model's constants live on the device that was current when it was
 *     created; qcl_sample_initial, qcl_propagate and qcl_propagate_batch
 *     must be called with that device current (INVALID_ARG otherwise).
 */
#ifndef QCL_H
#define QCL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QCL_MAX_STATES 8
#define QCL_MAX_MODES 128
#define QCL_MAX_MODES_MANY 32  /* mode limit of models with more than 4 states */
/* Walkers per reduction tile: the partial sums are kept per tile of this
 * many consecutive walkers. */
#define QCL_TILE 256

typedef enum {
    QCL_OK = 0,
    QCL_ERR_INVALID_ARG = 1,   /* bad size, pointer, value or layout */
    QCL_ERR_UNSUPPORTED = 2,   /* valid request this build cannot run */
    QCL_ERR_OUT_OF_MEMORY = 3, /* qcl_create_model could not allocate */
    QCL_ERR_DEVICE = 4,        /* a HIP call or kernel launch failed */
    QCL_ERR_NONFINITE = 5      /* qcl_reduce_observables: walkers with a
                                  non-finite weight or phase were excluded
                                  from the sums (the results are written;
                                  qcl_last_error() states the count) */
} qcl_status;

typedef enum {
    QCL_FP64 = 0,        /* everything in binary64 */
    QCL_FP32_ACC64 = 1   /* q, p, frame and per-step arithmetic in binary32;
                            weight, phase integral, near-degenerate
                            eigen-solves and all sums in binary64 */
} qcl_precision;

typedef enum {
    QCL_INIT_DIABATIC = 0, /* |k><k| in the diabatic basis */
    QCL_INIT_ADIABATIC = 1 /* |k><k| in the adiabatic basis */
} qcl_init_basis;

typedef enum {
    /* stay with probability 1/(1+S), move to candidate k with probability
     * |f_k|/(1+S); w <- w (1+S) sgn(f_k) (sgn = 1 when staying) */
    QCL_TRANS_NORMALIZED = 0,
    /* when S < 1: move to k with probability |f_k| (w <- w sgn f_k), else
     * stay with w <- w/(1-S); steps with S >= 1 use the normalized rule
     * and set QCL_FLAG_FALLBACK */
    QCL_TRANS_LINEAR = 1
} qcl_transition;

/* per-walker diagnostic bits (qcl_ensemble.flags) */
#define QCL_FLAG_NONFINITE 1u   /* w or Phi not finite: walker excluded from sums */
#define QCL_FLAG_DEGENERATE 2u  /* an adiabatic gap below DBL_MIN was met */
#define QCL_FLAG_RESOLVED64 4u  /* binary32 path met a gap below the model threshold and
                                   treated it in binary64 (N = 2: closed form re-evaluated;
                                   N > 2: closest pair re-rotated) */
#define QCL_FLAG_FALLBACK 8u    /* linear rule fell back to the normalized one */

typedef struct qcl_model_s *qcl_model; /* opaque, library-owned, immutable */

/* Model description (host pointers, read during qcl_create_model only). */
typedef struct {
    int32_t n_states;     /* N, 2 .. QCL_MAX_STATES (N > 4: linear models
                             with at most QCL_MAX_MODES_MANY modes) */
    int32_t n_modes;      /* M, 1 .. QCL_MAX_MODES */
    const double *mass;   /* [M], > 0 */
    const double *omega;  /* [M], > 0 */
    const double *v0;     /* [N*N] row-major, symmetric to 1e-12 relative */
    const double *k;      /* [M*N*N] row-major per mode, each symmetric */
    double hbar;          /* > 0 (1 in reduced units or eV-based units) */
} qcl_model_desc;

/* Initial state (Sec. II.A: partial Wigner transform of the nuclei).
 * Each mode j is drawn from the thermal Wigner distribution of its
 * harmonic well, centred on (q0_j, 0):
 *   var q = hbar/(2 m w tanh(hbar w/2kT)),  var p = hbar m w/(2 tanh(.)),
 * (kT = 0: ground state).  DIABATIC k: element (a,b) drawn with
 * probability |U_ka U_kb|/Z, Z = (sum_a |U_ka|)^2, w = sgn(U_ka U_kb) Z;
 * ADIABATIC k: (a,b) = (k,k), w = 1.  Phi = 0. */
typedef struct {
    double kT;            /* >= 0, finite */
    const double *q0;     /* [M] host */
    int32_t state;        /* k in 0 .. N-1 */
    int32_t basis;        /* qcl_init_basis */
} qcl_init_desc;

/* Walker ensemble: structure-of-arrays in device memory, owned by the
 * caller.  Every per-walker array has leading dimension ld (>= n_traj,
 * a multiple of 64); walker t of mode j lives at q[j*ld + t].  "real" is
 * double for QCL_FP64 and float for QCL_FP32_ACC64. */
typedef struct {
    int64_t n_traj;       /* walkers, >= 0 */
    int64_t ld;           /* leading dimension */
    int64_t traj_offset;  /* global id of walker 0 (random streams are keyed
                             by global id, so a slice reproduces the whole) */
    int64_t step;         /* global step counter; qcl_propagate advances it */
    int32_t prec;         /* qcl_precision */
    int32_t reserved;
    void *q;              /* device real [M][ld]  coordinates */
    void *p;              /* device real [M][ld]  momenta */
    void *u;              /* device real [N*N][ld] adiabatic frame:
                             u[(i*N + k)*ld + t] = U_ik, column k is the
                             eigenvector of the k-th lowest energy */
    double *w;            /* device [ld] weight */
    double *phase;        /* device [ld] Phi */
    uint8_t *a;           /* device [ld] element row */
    uint8_t *b;           /* device [ld] element column */
    uint32_t *flags;      /* device [ld] QCL_FLAG_* bits, or NULL */
} qcl_ensemble;

/* Propagation request. */
typedef struct {
    double dt;            /* > 0 */
    int32_t n_steps;      /* >= 0 */
    int32_t cadence;      /* >= 1: bin o receives global step o*cadence */
    int32_t n_out;        /* bins held by the partials buffer; every bin
                             reached by this call must be < n_out */
    int32_t scheme;       /* qcl_transition */
    uint64_t seed;        /* Philox key */
    int32_t occupancy;    /* register budget of the general kernels: 0 = the
                             compiler's choice; 3 = at most a third of the
                             register file per wave (3 waves per SIMD), for
                             binary32 ensembles of linear models with N > 2
                             or M > 8 and at most 32 modes; 2 = at most half
                             of it (2 waves per SIMD) for such models with
                             33..64 modes (other models ignore both).
                             The result is bitwise the same either way; the
                             faster choice depends on the model (see the
                             tuner in the Python package). */
    int32_t workgroups_per_cu; /* qcl_propagate_batch: workgroups each compute
                             unit receives in the item's persistent launch,
                             0 = as many as fit, 1..32 = at most that many
                             (items that differ in it launch separately);
                             qcl_propagate ignores it.  Results are bitwise
                             the same for every value. */
} qcl_prop_desc;

/* Builds a model: validates the description, derives the per-mode
 * constants and uploads them to the current device (a few KB, owned by
 * the model).  Errors: INVALID_ARG (sizes, non-finite values, mass/omega
 * <= 0, asymmetry), OUT_OF_MEMORY, DEVICE. */
qcl_status qcl_create_model(const qcl_model_desc *desc, qcl_model *out);

/* Higher separable powers of each mode (beyond the linear-vibronic form;
 * Eq. 1 holds for any V(R), and the paper's closing section names general
 * potentials as the next step): the model's potential becomes
 *   V(q) = V0 + sum_j [ q_j K_j + sum_{k=2..degree} q_j^k A_jk ],
 * so the adiabatic forces and couplings use
 *   dV/dq_j = K_j + sum_k k q_j^(k-1) A_jk.
 * k = 2 gives state-dependent frequencies, k = 3, 4 anharmonicity.  The
 * Wigner initial state stays that of the harmonic wells (m_j, w_j). */
typedef struct {
    int32_t degree;       /* highest power, 2 .. 4 */
    int32_t reserved;
    const double *a;      /* host [M][degree-1][N][N] row-major: A_jk for
                             k = 2..degree, each symmetric to 1e-12 */
} qcl_poly_desc;

/* As qcl_create_model, with the higher powers of poly (read during the
 * call only).  Two-state models with at most 8 modes run on the two-state
 * closed-form kernels; the others on the general-N kernels with every
 * coupling direction kept (rank padded to N(N+1)/2).  Both use the default
 * register budget (qcl_prop_desc.occupancy is ignored).
 * Errors: as qcl_create_model; INVALID_ARG also for degree outside [2, 4],
 * a NULL poly->a, non-finite or asymmetric A_jk. */
qcl_status qcl_create_model_poly(const qcl_model_desc *desc, const qcl_poly_desc *poly, qcl_model *out);

#define QCL_MAX_PAIRS 64         /* bilinear terms per model (see qcl_create_model_bilinear) */
#define QCL_MAX_MODES_BILINEAR 32

/* Cross-mode bilinear terms (the same extension of Eq. 1's potential as
 * qcl_poly_desc, with couplings between two modes, e.g. the Duschinsky
 * mixing of a quadratic vibronic-coupling model):
 *   V(q) += sum_p q_{i_p} q_{j_p} B_p,   dV/dq_i += q_j B_p, dV/dq_j += q_i B_p.
 * The Wigner initial state stays that of the harmonic wells (m_j, w_j). */
typedef struct {
    int32_t n_pairs;      /* 1 .. QCL_MAX_PAIRS */
    int32_t reserved;
    const int32_t *pairs; /* host [n_pairs][2]: modes (i, j), 0 <= i, j < M, i != j */
    const double *b;      /* host [n_pairs][N][N] row-major: B_p, each symmetric to 1e-12 */
} qcl_bilinear_desc;

/* As qcl_create_model_poly (poly may be NULL: no powers above 1), with the
 * bilinear terms of bil (read during the call only).  Such a model runs on
 * the general-N kernels for N = 2..4 (also N = 2), every coupling direction
 * kept; qcl_model_degree reports at least 2.  On the device the terms
 * become squared mode combinations y_s = c_s . q, with slot weights: either
 * each term split exactly as q_i q_j = ((q_i + q_j)^2 - (q_i - q_j)^2) / 4
 * (two combinations, coefficients +-1), or, when that needs fewer, the
 * eigendecomposition of each coupling slot's M x M matrix (one combination
 * per nonzero eigenvalue; dense couplings among a few modes, or mode mixing
 * shared by the states).  At most 16 combinations, and at most 16 modes
 * when more than 8 are needed.
 * Errors: as qcl_create_model_poly; INVALID_ARG also for a NULL bil, pairs
 * or b, n_pairs outside [1, QCL_MAX_PAIRS], a mode index out of range or
 * i == j, non-finite or asymmetric B_p; UNSUPPORTED for more than 4 states,
 * more than QCL_MAX_MODES_BILINEAR modes, more than 16 combinations, or
 * more than 16 modes with more than 8 combinations. */
qcl_status qcl_create_model_bilinear(const qcl_model_desc *desc, const qcl_poly_desc *poly,
                                     const qcl_bilinear_desc *bil, qcl_model *out);

/* Number of bilinear terms of a model (0 for NULL or none). */
int32_t qcl_model_pairs(qcl_model model);

/* A model with a supplied potential.  Eq. 1 holds for any potential
 * V(R), and the paper's closing section (Sec. IV) names on-the-fly
 * potentials, forces and couplings (molecular dynamics, QM/MM) as the next
 * step; this entry point takes the diabatic potential matrix as device
 * source code, compiled for the current device with the library's kernels
 * when the model is built (hipRTC).  The Hamiltonian is
 *   H = sum_j p_j^2 / (2 m_j) + V(q),
 * V(q) a real symmetric N x N matrix holding every q-dependent term (the
 * nuclear potential on its diagonal too).  The source defines three
 * binary64 device functions, in the global namespace:
 *
 *   __device__ void qcl_potential(const double *q, double *V);
 *       V[s], s = 0 .. N(N+1)/2 - 1: V_kl (k <= l) at q, row by row
 *   __device__ void qcl_force(const double *q, const double *w, double *f);
 *       f[j] = -sum_s w[s] dV_s/dq_j, j = 0 .. M-1
 *   __device__ void qcl_coupling(const double *q, const double *v, double *K);
 *       K[s] = sum_j v[j] dV_s/dq_j
 *
 * and may use QCL_N, QCL_M (integer constants) and qcl_param[i] (the
 * given parameter values, compile-time constants).  The kernels call
 * qcl_force with the slot weights of a walker's element (a, b), giving the
 * mean force -[(U^T dV/dq_j U)_aa + (U^T dV/dq_j U)_bb] / 2, and
 * qcl_coupling with v = p/m, giving D = U^T K U for the Monte Carlo move.
 * The three must agree (f and K are contractions of the same gradient).
 * The program is compiled without contraction of separate multiplies and
 * adds (write fma() where a fused operation is wanted), so that a run split
 * over calls reproduces the uninterrupted one bit for bit.
 * desc supplies N (2..4), M (1..QCL_MAX_MODES_SOURCE), the masses, hbar and
 * the frequencies omega of the harmonic reference that the Wigner initial
 * state is drawn from (qcl_sample_initial); v0 and k are not read.  A
 * source that also defines the three functions for float arguments
 * (overloads or templates) and defines QCL_SOURCE_FP32 gets binary32
 * kernels too (binary32 state and step; binary64 weight, phase and sums;
 * where the smallest gap falls below 1e-4 of the largest hbar*omega, the
 * closest pair re-solved from the binary64 potential); otherwise binary32
 * ensembles are UNSUPPORTED.  In qcl_propagate_batch the items of one such
 * model form a class of their own (its compiled program holds persistent
 * batched kernels).  Errors: INVALID_ARG (as qcl_create_model
 * for the sizes and the masses and frequencies; NULL source; n_params
 * outside [0, QCL_MAX_PARAMS] or a non-finite parameter; a source that does
 * not compile, with the compiler's log in qcl_last_error), DEVICE (no
 * usable device, or the compiled code does not load). */
#define QCL_MAX_MODES_SOURCE 32
#define QCL_MAX_PARAMS 256
typedef struct {
    const char *source;    /* NUL-terminated device source (host) */
    const double *params;  /* [n_params] host, or NULL when n_params is 0 */
    int32_t n_params;
    int32_t reserved;
} qcl_source_desc;

qcl_status qcl_create_model_source(const qcl_model_desc *desc, const qcl_source_desc *src, qcl_model *out);

/* 1 when the model was built by qcl_create_model_source, else 0. */
int32_t qcl_model_is_source(qcl_model model);

/* Highest power of q_j in the model's potential: 1 for a linear-vibronic
 * model, 2..4 for one built by qcl_create_model_poly (at least 2 for one
 * built by qcl_create_model_bilinear), 0 for NULL. */
int32_t qcl_model_degree(qcl_model model);

/* Frees a model (NULL is accepted).  Work that uses it must be complete. */
qcl_status qcl_destroy_model(qcl_model model);

int32_t qcl_model_states(qcl_model model);
int32_t qcl_model_modes(qcl_model model);
/* Rank of the mode couplings: the number of orthonormal directions B_r with
 * K_j = sum_r C_jr B_r that qcl_create_model found (0 when every K_j is 0;
 * 0 for a NULL model). */
int32_t qcl_model_rank(qcl_model model);

/* Layout of one ensemble in a single caller allocation: *ld is the
 * leading dimension and *bytes the size of a buffer that
 * qcl_ensemble_bind() carves into the arrays above (256-byte aligned
 * sub-buffers; flags included). */
qcl_status qcl_ensemble_bytes(qcl_model model, int64_t n_traj, int32_t prec,
                              int64_t *ld, size_t *bytes);

/* Fills *ens with pointers into base (device, >= qcl_ensemble_bytes,
 * 256-byte aligned); sets step = 0, traj_offset as given. */
qcl_status qcl_ensemble_bind(qcl_model model, void *base, int64_t n_traj, int32_t prec,
                             int64_t traj_offset, qcl_ensemble *ens);

/* Bytes of the partial-sum buffer for n_traj walkers and n_out bins:
 * n_tiles = ceil(n_traj/QCL_TILE) rows of n_out x (2 x N x N x 4 + 1)
 * doubles (per bin the sums of Re, Im, Re^2, Im^2 of every adiabatic and
 * diabatic element, then the number of walkers excluded from the bin),
 * plus scratch rows and n_out excluded counts used by
 * qcl_reduce_observables. */
qcl_status qcl_partials_bytes(qcl_model model, int64_t n_traj, int32_t n_out, size_t *bytes);

/* Samples the initial ensemble (Sec. II.A, partial Wigner transform) and
 * writes bin 0 of the partials.  Random numbers: Philox4x32-10 keyed by
 * seed, counter (gid lo, gid hi, j, 1) for mode j and (gid lo, gid hi, 0,
 * 2) for the element draw, gid = traj_offset + walker index.  Sampling is
 * done in binary64 and stored in the ensemble's precision.
 * partials: device, qcl_partials_bytes(model, n_traj, n_out).  Sets
 * ens->step = 0.  Errors: INVALID_ARG, DEVICE. */
qcl_status qcl_sample_initial(qcl_model model, const qcl_init_desc *init, uint64_t seed,
                              qcl_ensemble *ens, double *partials, int32_t n_out, void *stream);

/* Advances every walker prop->n_steps steps from global step ens->step
 * (Eq. 1; Sec. II.B: one fixed ensemble, no spawning).  Step n:
 *   1. Monte Carlo move at (q_n, p_n): candidates (c,b), c != a, with
 *      f = dt v.d_ac, then (a,c), c != b, with f = dt v.d_bc, where
 *      v.d_ab = [U^T (sum_j p_j/m_j K_j) U]_ab / (E_b - E_a);
 *      u = Philox(seed; gid lo, gid hi, n>>2, 0) word n&3 as
 *      (2 floor(x/2^9) + 1) 2^-24; p is not changed;
 *   2. velocity Verlet with the mean force of the new element,
 *      F_j = -m_j w_j^2 q_j - [(U^T K_j U)_aa + (U^T K_j U)_bb]/2;
 *      eigen-solve at q_{n+1} (energies ascending, each eigenvector's sign
 *      kept continuous with the previous frame);
 *   3. Phi += dt [w_ab(q_n) + w_ab(q_{n+1})]/2;
 *   4. if (n+1) % cadence == 0: bin (n+1)/cadence of the partials.
 * Then ens->step += n_steps.  The result does not depend on how the steps
 * are split over calls.  Errors: INVALID_ARG (including a bin >= n_out),
 * UNSUPPORTED, DEVICE. */
qcl_status qcl_propagate(qcl_model model, qcl_ensemble *ens, const qcl_prop_desc *prop,
                         double *partials, void *stream);

/* One instance of a batched propagation: the arguments of one
 * qcl_propagate call. */
typedef struct {
    qcl_model model;
    qcl_ensemble *ens;    /* host struct; ens->step is advanced */
    qcl_prop_desc prop;
    double *partials;     /* device, as for qcl_propagate */
} qcl_batch_item;

/* Device workspace needed by qcl_propagate_batch for these items (0 when
 * no item has work).  Errors: as qcl_propagate_batch's validation. */
qcl_status qcl_batch_workspace_bytes(const qcl_batch_item *items, int32_t n_items, size_t *bytes);

/* Propagates many independent ensembles (Sec. II.B: the walkers of every
 * instance are independent, so instances of different size, model and
 * length can share the device).  The result of every item is bitwise the
 * one qcl_propagate would give for it alone.
 *
 * Items that need the same kernel (two-state closed form with the same
 * mode count; or the same state count N and padded mode count; or the same
 * model with a supplied potential; same precision and transition rule)
 * form one class.  Each class runs as ONE
 * persistent launch (about one workgroup per free slot of the device);
 * its workgroups take (item, tile of QCL_TILE walkers) pairs from a device
 * counter, heaviest tiles first, so uneven instances balance across the
 * device.  Several classes run concurrently on internal streams forked
 * from the given stream and joined back into it (the call stays ordered on
 * the given stream); the first call with more than one class on a device
 * creates those streams and their events, which live until the process
 * ends.
 *
 * workspace: device, >= qcl_batch_workspace_bytes(items, n_items),
 * 256-byte aligned; holds the descriptors and counters and is written by
 * the call (no host buffer is kept).  Calls whose execution overlaps on
 * the device must use different workspaces.  An ensemble or partials
 * buffer may appear in one item only.  Errors: INVALID_ARG (any item
 * invalid as for qcl_propagate, a shared ensemble, a small or misaligned
 * workspace), UNSUPPORTED, DEVICE; nothing is launched and no step
 * counter changes unless every item is valid. */
qcl_status qcl_propagate_batch(const qcl_batch_item *items, int32_t n_items, void *workspace,
                               size_t workspace_bytes, void *stream);

/* Size of the library's own per-device workspace used by
 * qcl_propagate_batch_static: room for the descriptors of about 2000
 * batch items (each GPU the library runs on holds it until the process
 * ends). */
#define QCL_STATIC_WORKSPACE_BYTES (4u << 20)

/* qcl_propagate_batch for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same propagation, bitwise, with the descriptors and tile
 * counters in a library-owned static device array of
 * QCL_STATIC_WORKSPACE_BYTES per device instead of a caller workspace.  It
 * calls no hipMalloc, hipFree or other device allocation; its classes run
 * one after another on the given stream (no side streams).  Every call on a
 * device rewrites that device's array (descriptors and zeroed counters);
 * calls whose execution overlaps on one device race on it, so they must be
 * ordered (one stream, or events).  Errors: as qcl_propagate_batch;
 * INVALID_ARG also when the batch's descriptors exceed
 * QCL_STATIC_WORKSPACE_BYTES (qcl_batch_workspace_bytes gives the size
 * needed), DEVICE when the array's address cannot be obtained. */
qcl_status qcl_propagate_batch_static(const qcl_batch_item *items, int32_t n_items, void *stream);

/* Ensemble averages (Sec. II.B: deterministic-order reduction).  Sums the
 * tile partials over tiles in a fixed pairwise tree and writes, to device
 * memory out [n_out][2][N][N][4]:
 *   [o][0][a][b] adiabatic rho_ab, [o][1][i][j] diabatic rho_ij, each as
 *   (mean Re, mean Im, standard error Re, standard error Im) over n_traj
 *   walkers (normalised by n_traj; SE = sqrt((S2 - S1^2/T)/(T(T-1)))).
 * A walker whose weight or phase is not finite (the sign problem, Sec. I,
 * can drive |w| past the binary64 range) contributes zeros from the first
 * bin it is non-finite at, and is counted per bin.  This call waits for the
 * reduction to finish on the stream and returns QCL_ERR_NONFINITE when any
 * bin excluded a walker, with the largest count and its bin in
 * qcl_last_error(); out is written either way.  n_traj must be the walker
 * count the partials were sized for (n_traj >= 1); the partials are read,
 * not modified (their scratch rows and counts are).
 * Errors: INVALID_ARG, DEVICE, NONFINITE. */
qcl_status qcl_reduce_observables(qcl_model model, double *partials, int64_t n_traj,
                                  int32_t n_out, double *out, void *stream);

/* The same reduction without waiting: enqueues it on the stream and
 * returns.  When excluded is not NULL it receives the per-bin counts of
 * excluded walkers (device int64 [n_out], 256-byte aligned).
 * Errors: INVALID_ARG, DEVICE (never NONFINITE). */
qcl_status qcl_reduce_observables_async(qcl_model model, double *partials, int64_t n_traj,
                                        int32_t n_out, double *out, int64_t *excluded, void *stream);

/* Fixed-budget resampling between propagation calls (the paper's CPU code
 * spawned walkers and let their number grow, Sec. II.B; this keeps T).
 * The T walkers of src are replaced in dst by T copies drawn by systematic
 * resampling in proportion to |w|, decided in exact integer arithmetic:
 *   k_i = ceil(|w_i| / w_max * 2^32) for walkers with finite nonzero w and
 *         finite phase (else 0; w_max over those walkers),
 *   P_i = k_0 + ... + k_{i-1}, K = P_T,
 *   output j copies the source i with P_i <= X_j < P_{i+1},
 *   X_j = floor((j 2^32 + U) K / (T 2^32)), U = word 0 of Philox4x32-10 with
 *   key (seed lo, seed hi) and counter (traj_offset lo, traj_offset hi,
 *   step lo, 3),
 * and output j gets the weight w_i * (K / (T k_i)) (binary64), so every
 * walker's expected contribution is unchanged.  The rest of the state is
 * copied; output j continues with the random stream of global id
 * traj_offset + j.  If K = 0 the ensemble is copied unchanged.
 * src and dst: same model, precision, n_traj (< 2^31), ld and traj_offset;
 * no array shared between them.  dst->step is set to src->step; src is not
 * changed.  workspace: device memory of qcl_resample_workspace_bytes bytes,
 * 256-byte aligned, caller-owned (contents undefined afterwards).  Errors:
 * INVALID_ARG, DEVICE.  Asynchronous on stream. */
qcl_status qcl_resample_workspace_bytes(int64_t n_traj, size_t *bytes);
qcl_status qcl_resample(qcl_model model, const qcl_ensemble *src, qcl_ensemble *dst, uint64_t seed,
                        void *workspace, size_t workspace_bytes, void *stream);

/* Thread-local description of the last failure on this thread. */
const char *qcl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QCL_H */
