/*
 * soap.h -- C ABI of the MI355X (gfx950) separable-SOAP / GAP library.
 *
 * Method: M. A. Caro, "Optimizing many-body atomic descriptors for enhanced
 * computational performance of machine learning based interatomic potentials",
 * arXiv:1905.02142 (2019).  Section and equation numbers below refer to it.
 *
 * What the library computes, for every atom i of one or many periodic structures:
 *   - the neighbours j (with lattice image T) inside the cutoff sphere (Sec. I);
 *   - the separable-density expansion coefficients c_nlm (Eqs. (05), (08)) from
 *     the analytic radial overlaps of Sec. III.A (Eqs. (19), (02), (04) and the
 *     Gaussian-basis closed form), the ilexp factors and spherical harmonics of
 *     Sec. III.C, summed over neighbours;
 *   - the power spectrum p_{nn'l} (Eq. (09)) and the unit descriptor q = p/|p|;
 *   - the GAP local energies e_i = sum_s alpha_s (q_i . q_s)^zeta (Sec. IV.A),
 *     forces F = -dE/dr and dE/dalpha_s (not in the paper: derived adjoints).
 *
 * Conventions
 *   - Every array argument is a DEVICE pointer owned by the caller unless it is
 *     marked (host).  Arrays are row-major and contiguous.  The library never
 *     frees caller memory.
 *   - All device work is enqueued on the given stream in stream order.  Entry
 *     points return after enqueueing, except where a host read-back is stated.
 *   - Errors are returned as soap_status; nothing is thrown across the ABI.
 *     Argument errors are detected on the host before anything is enqueued and
 *     leave outputs untouched.  A HIP launch failure returns SOAP_EHIP;
 *     asynchronous device faults surface at the next synchronising call.
 *     soap_last_error() gives a message for the most recent failure on a context.
 *   - Units: positions and lengths in Angstrom; energies in the units of alpha;
 *     forces = -dE/dr in energy units per Angstrom.
 *   - A context is not thread safe: calls on one context must not overlap in
 *     time (they may use different streams if the caller orders them).
 */
#ifndef SOAP_H
#define SOAP_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SOAP_OK = 0,
  SOAP_EINVAL = -1,     /* invalid argument (checked on the host) */
  SOAP_ENOMEM = -2,     /* device allocation of the context workspace failed */
  SOAP_EOVERFLOW = -3,  /* neighbour list capacity too small; see required_pairs */
  SOAP_EHIP = -4,       /* a HIP runtime call failed */
  SOAP_ENOTSUP = -5     /* valid but unsupported combination */
} soap_status;

/* Arithmetic of the GAP kernel contraction (S = Q Q_s^T and Qbar = G Q_s).
 * The exp/erf terms are FP64 in every mode, the radial recursion and the
 * orthonormal transform W are FP64 or double-double (soap_radial_precision);
 * c_nlm is FP64 in every mode, p and q are FP64 except in SOAP_MIXED_BF16_PS. */
typedef enum {
  SOAP_FP64 = 0,        /* FP64 MFMA */
  SOAP_MIXED_F32 = 1,   /* FP32 operands, FP32 accumulation (MFMA) */
  SOAP_MIXED_BF16 = 2,  /* BF16 operands, FP32 accumulation (MFMA) */
  SOAP_MIXED_BF16X3 = 3, /* split-BF16 (hi/lo, three products), FP32 accumulation */
  SOAP_MIXED_BF16_PS = 4 /* BF16 GAP contractions as SOAP_MIXED_BF16, and the power spectrum
                            P_l = C_l C_l^T (Eq. (09)) and its adjoint cbar_l = M_l C_l on the
                            matrix cores in BF16 with FP32 accumulation (n_species n_max <= 48) */
} soap_precision;

/* Arithmetic of the radial stage (Sec. III.A): the integration-by-parts
 * recursion of Eq. (04) and b = W b_alpha.  The overlap matrix S of the basis is
 * nearly singular (smallest eigenvalue ~1e-11 at n_max = 8, ~1e-14 at 10, ~4e-18
 * at 12), so W = S^{-1/2} has entries up to ~1e5, ~5e6 and ~2e8 and multiplies
 * every rounding of b_alpha: in FP64 the per-pair b_n carry relative errors of
 * ~3e-11 (n_max = 8), ~1e-9 (10) and ~4e-8 (12).  In double-double the recursion
 * and W b_alpha (with W itself to 106 bits) hold b_n to ~1e-14 (10) and ~2e-13
 * (12); the erf and exp seeds stay FP64. */
typedef enum {
  SOAP_RADIAL_AUTO = 0, /* double-double when precision is SOAP_FP64 and n_max >= 8, else FP64 */
  SOAP_RADIAL_FP64 = 1,
  SOAP_RADIAL_DD = 2
} soap_radial_precision;

/* Hyper-parameters: Eq. (15) and Sec. III.B.  Defaults in brackets. */
typedef struct {
  int n_max;             /* radial basis size, 2..12: n_max-1 polynomials + 1 Gaussian */
  int l_max;             /* 0..12 */
  int n_species;         /* >= 1; neighbours of species s fill channels s*n_max..s*n_max+n_max-1 */
  double r_cut;          /* hard cutoff r_hard (> 0) */
  double r_soft;         /* soft cutoff; == r_cut means no buffer zone [r_cut] */
  double n_f;            /* buffer-zone filter parameter [4.0] */
  double sigma0_r;       /* radial width at r = 0 (> 0) */
  double sigma0_perp;    /* angular width at r = 0 (> 0) */
  double alpha_r;        /* d sigma_r / dr (>= 0) [0] */
  double alpha_perp;     /* d sigma_perp / dr (>= 0) [0] */
  double a;              /* amplitude exponent of (1 + 2x^3 - 3x^2)^a (>= 0) [0] */
  double central_weight; /* weight of the central-atom Gaussian; 0 drops it [1.0] */
  int l_weight;          /* 0: factor 2l+1 of Eq. (08) as printed [0]; 1: factor 1 */
  soap_precision precision; /* GAP contraction arithmetic [SOAP_FP64] */
  soap_radial_precision radial_precision; /* radial stage arithmetic [SOAP_RADIAL_AUTO] */
} soap_params;

/* Opaque context: owns the basis tables (W = S^{-1/2} computed on the host in
 * 113-bit arithmetic, then rounded) and a device workspace that grows on demand. */
typedef struct soap_ctx soap_ctx;

/* Neighbour list in CSR form, all arrays caller-allocated DEVICE memory.
 * Centre atom i owns pairs offsets[i] .. offsets[i+1]-1 in a fixed order
 * (neighbouring cell-list bins in a fixed sequence, atoms by index inside a
 * bin), the same on every build of the same input.
 * For pair p: j[p] neighbour atom, (dx,dy,dz)[p] = r_j + T - r_i, img[p] the
 * lattice image T packed as ((Tx+512) << 20 | (Ty+512) << 10 | (Tz+512)),
 * rev[p] the index of the reverse pair (j -> i, -T), center[p] = i.
 * Capacities: offsets n_atoms+1; all per-pair arrays `capacity` entries. */
typedef struct {
  int n_atoms;
  int n_structures;
  long long n_pairs;     /* written by soap_build_neighbors; SOAP_PAIRS_DEFERRED after
                            soap_build_neighbors_async (the count is offsets[n_atoms]) */
  long long capacity;    /* set by the caller */
  int32_t* offsets;
  int32_t* j;
  int32_t* img;
  int32_t* rev;
  int32_t* center;
  double* dx;
  double* dy;
  double* dz;
} soap_nlist;

/* n_pairs of a list whose pair count is still on the device only.  The entry
 * points accept such a list: they size their work by `capacity` and every
 * kernel reads min(offsets[n_atoms], capacity) pairs and cuts each atom's range
 * at the capacity, so they never touch memory beyond it, even when the build
 * overflowed (the results are then meaningless; soap_neighbors_check says so). */
#define SOAP_PAIRS_DEFERRED (-1LL)

/* Validate `p` and build the basis tables.  Returns SOAP_EINVAL for n_max
 * outside 2..12, l_max outside 0..12, n_species < 1, non-positive r_cut or
 * widths, r_soft outside (0, r_cut], n_f <= 0, negative alpha_r, alpha_perp or
 * a, l_weight not 0/1, or an unknown precision or radial precision.  Needs a
 * current HIP device. */
soap_status soap_create(const soap_params* p /* host */, soap_ctx** out /* host */);
void soap_destroy(soap_ctx* ctx);

/* Descriptor length K = n_ch (n_ch + 1) / 2 * (l_max + 1), n_ch = n_species * n_max. */
int soap_descriptor_dim(const soap_ctx* ctx);
const char* soap_status_string(soap_status s);
const char* soap_last_error(const soap_ctx* ctx);

/*
 * Neighbour list (Sec. I: all atoms inside the cutoff sphere, every periodic
 * image counted separately, self-images included, the centre itself excluded):
 * all (i, j, T) with 0 < |r_j + T - r_i| < r_cut, T a lattice vector of i's
 * structure on its periodic axes, j in the same structure.
 *   pos            n_atoms x 3 positions (device)
 *   cells          n_structures x 3 x 3, rows are lattice vectors (host)
 *   pbc            n_structures x 3, nonzero = periodic axis (host)
 *   struct_offsets n_structures + 1 atom offsets (host); NULL means one structure
 *   nl             in: capacity and arrays; out: n_pairs and the arrays
 *   required_pairs (host, nullable) receives the pair count
 * Reads the pair count back to the host (one stream synchronisation, after the
 * whole build is enqueued).  If it exceeds nl->capacity, returns
 * SOAP_EOVERFLOW, sets *required_pairs to the count and nl->n_pairs to 0, and
 * leaves the per-pair arrays undefined.  Coincident atoms (distance < 1e-8) or
 * non-finite positions return SOAP_EINVAL.
 */
soap_status soap_build_neighbors(soap_ctx* ctx, int n_atoms, const double* pos, const double* cells,
                                 const int32_t* pbc, const int32_t* struct_offsets, int n_structures,
                                 soap_nlist* nl, long long* required_pairs, hipStream_t stream);

/*
 * The same build with no host synchronisation, for steps that must not stall
 * the host (and for stream capture into a HIP graph): every kernel is enqueued
 * on `stream`; the pair count stays on the device at offsets[n_atoms], and
 * nl->n_pairs is set to SOAP_PAIRS_DEFERRED.  Pairs are written only below
 * nl->capacity, so an undersized list is safe but holds an incomplete result.
 * Host-side argument errors are returned at once; device-side findings
 * (overflow, non-finite or coincident positions) are reported by
 * soap_neighbors_check.  Under stream capture the structure geometry must equal
 * that of the previous build on this context (its upload is not captured), and
 * the workspace must already be large enough (an earlier call outside capture).
 */
soap_status soap_build_neighbors_async(soap_ctx* ctx, int n_atoms, const double* pos, const double* cells,
                                       const int32_t* pbc, const int32_t* struct_offsets, int n_structures,
                                       soap_nlist* nl, hipStream_t stream);

/*
 * Waits for `stream` and reports the most recent build on this context into
 * `nl`: *n_pairs (host, nullable) receives the pair count; returns SOAP_OK,
 * SOAP_EOVERFLOW if the count exceeds nl->capacity, or SOAP_EINVAL for
 * non-finite or coincident positions (the same checks as soap_build_neighbors).
 * nl is not modified.
 */
soap_status soap_neighbors_check(soap_ctx* ctx, const soap_nlist* nl, long long* n_pairs, hipStream_t stream);

/*
 * Descriptors q (n_atoms x K, FP64) of every atom of `nl`, and |p| (n_atoms,
 * nullable).  Defined by Eq. (08) (c_nlm summed over the neighbours, with the
 * radial coefficients of Sec. III.A and the angular factors of Sec. III.C),
 * Eq. (09) (the power spectrum p_{nn'l}, here over species channels) and the
 * normalisation q = p / |p| of Sec. I; q_i is packed as channel pairs a <= b
 * (a outer), then l, with the factor sqrt(2) on a != b so that the packed norm
 * equals the full one.  species: n_atoms labels in 0..n_species-1 (an atom with another
 * label contributes to no density; with n_species = 1 the labels are not read).
 * Atoms with p = 0 get q = 0.  The coefficients c_nlm are kept in the context for a following
 * soap_descriptor_grad / gap_energy_forces call on the same list.
 */
soap_status soap_descriptor(soap_ctx* ctx, const soap_nlist* nl, const int32_t* species, double* q,
                            double* p_norm, hipStream_t stream);

/*
 * soap_descriptor for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation): the
 * same results, bit for bit, from the same kernels, but every intermediate
 * buffer (the per-pair fields, c_nlm, the central-atom factors and |p| when
 * p_norm is NULL) lives in one fixed array of SOAP_NOALLOC_SCRATCH_BYTES that
 * the library holds on each device for the life of the process.  The call makes
 * no device allocation, free or copy and does not grow the context's workspace;
 * the caller still passes q (and p_norm) and the neighbour list.
 * Limits and errors: the buffers take 8 ROW 64 ceil(P / 64) bytes for P pairs
 * (P = nl->capacity while the count is deferred), 8 n_species NB ((l_max+1)^2 + 1)
 * bytes per atom, 96 bytes and, with p_norm NULL, 8 bytes per atom, each rounded
 * up to 256 bytes, where ROW and NB come from the compiled basis bucket (ROW = 56,
 * NB = 8 at n_max = l_max = 8; ROW = 68, NB = 10 at 10): 4096 atoms with 211,320
 * pairs at n_max = l_max = 8 take 116 MB.  A call needing more than
 * SOAP_NOALLOC_SCRATCH_BYTES returns SOAP_ENOTSUP before
 * any device work, with the sizes in soap_last_error; SOAP_EINVAL as
 * soap_descriptor, or when the current device is not the context's; SOAP_EHIP if
 * the scratch array's address could not be looked up at soap_create.
 * Every call on one device shares that device's array and leaves its contents
 * behind: calls that overlap in time on one device (other streams, other
 * contexts, other threads) race and must be ordered by the caller.
 */
#define SOAP_NOALLOC_SCRATCH_BYTES (128LL << 20)
soap_status soap_descriptor_noalloc(soap_ctx* ctx, const soap_nlist* nl, const int32_t* species, double* q,
                                    double* p_norm, hipStream_t stream);

/*
 * Vector-Jacobian product of the descriptor: pos_grad (n_atoms x 3) +=
 * sum_i (dq_i/dr)^T q_bar_i, with q_bar (n_atoms x K) in the packing of
 * soap_descriptor.  The derivative of the chain Eq. (08) -> Eq. (09) -> q = p/|p|
 * with respect to the atomic positions (the paper gives the forward maps only;
 * the kernel derivatives it reports missing in Sec. IV.A are built on this
 * product).  Invalid arguments: SOAP_EINVAL (null species, q_bar or pos_grad with
 * n_atoms > 0), SOAP_ENOTSUP (a descriptor too large for one workgroup's LDS).
 * Recomputes c_nlm and the
 * per-pair radial/angular terms and their derivatives instead of storing a
 * per-pair Jacobian.  Deterministic: each atom gathers its pair terms in a
 * fixed order through the reverse-pair index.
 */
soap_status soap_descriptor_grad(soap_ctx* ctx, const soap_nlist* nl, const int32_t* species,
                                 const double* q_bar, double* pos_grad, hipStream_t stream);

/*
 * Descriptor Jacobian in tiles, for fitting with forces (the kernel derivatives
 * that Sec. IV.A reports the new SOAP code lacked): for the descriptor components
 * k0 <= k < k1,
 *   jac[((k - k0) * 3 + x) * B + p] = d q_{i,k} / d (d_p)_x
 * for every pair p of centre i, d_p = r_j + T - r_i, x = 0, 1, 2, where B is
 * nl->n_pairs (or nl->capacity for a list whose count is still on the device).
 * The derivative of q_i with respect to a position follows by the chain rule:
 * d/dr_j gains +jac_p, d/dr_i gains -jac_p.  jac: (k1 - k0) x 3 x B doubles
 * (device, caller-owned).  One forward pass, then one adjoint pass per
 * component (with qbar = the unit vector e_k on every atom).  SOAP_EINVAL unless
 * 0 <= k0 < k1 <= K.
 */
soap_status soap_descriptor_jacobian(soap_ctx* ctx, const soap_nlist* nl, const int32_t* species, int k0, int k1,
                                     double* jac, hipStream_t stream);

/*
 * GAP energies and forces.  The local energy of Sec. IV.A, e_i = sum_s alpha_s
 * k(q_i, q_s), with the dot-product kernel k = (q_i . q_s)^zeta of Sec. I
 * (no constant offset, no prefactor: both are absorbed into alpha); forces
 * F = -dE/dr through the derivative of the descriptor (as soap_descriptor_grad).
 * q_sparse: M x K sparse descriptors (FP64; cast by
 * the library to the context's precision), alpha: M weights, zeta >= 1 integer.
 * Outputs: e_atom (n_atoms) local energies; forces (n_atoms x 3, nullable =>
 * energies only) = -dE/dr, overwritten; alpha_grad (M, nullable) = dE/dalpha_s
 * = sum_i (q_i . q_s)^zeta, overwritten.  Computes the descriptor internally.
 * Errors: SOAP_EINVAL for M < 1, zeta < 1 (non-integer powers of the possibly
 * negative q_i . q_s are not defined) or null required pointers; SOAP_ENOTSUP
 * when the workspace would have to grow while `stream` is being captured.
 * Enqueues kernels only (no memset, copy or synchronisation), so a call whose
 * workspace is already large enough can be captured in a HIP graph.
 */
soap_status gap_energy_forces(soap_ctx* ctx, const soap_nlist* nl, const int32_t* species,
                              const double* q_sparse, const double* alpha, int M, int zeta,
                              double* e_atom, double* forces, double* alpha_grad, hipStream_t stream);

/* Host utility: the orthonormalisation table W = S^{-1/2} of the radial basis
 * (Sec. III.A) for these parameters, n_max x n_max row-major (host), and the
 * eigenvalues of S in ascending order (host, nullable).  S and W are formed in
 * binary128 and rounded once.  SOAP_EINVAL for invalid sizes or if S is not
 * positive definite. */
soap_status soap_radial_basis_table(int n_max, double r_cut, double sigma0_r, double* W, double* lambda);

/* Per-stage device timing.  soap_profile(ctx, 1) makes every later call record a
 * pair of hipEvents around each stage, on the stream that stage is launched
 * on; soap_profile(ctx, 0) stops recording.  soap_profile_stages(ctx, mask)
 * records only the stages whose bit (1 << stage) is set.  soap_profile_read
 * waits for the recorded events, writes per stage the summed milliseconds and
 * the number of launches (host arrays of SOAP_STAGE_COUNT entries) and clears
 * the record.  Recording adds two event records per timed stage.  Stages 1, 4,
 * 5, 7 and 9 are one kernel each. */
typedef enum {
  SOAP_STAGE_NEIGHBORS = 0,     /* cell list, pair count and fill, reverse index */
  SOAP_STAGE_DESCRIPTOR = 1,    /* c_nlm, power spectrum, q (one kernel) */
  SOAP_STAGE_GAP_SCORES = 2,    /* operand conversion, S = Q Q_s^T with the zeta epilogue: e, G, dE/dalpha */
  SOAP_STAGE_GAP_QBAR = 3,      /* Qbar = G Q_s */
  SOAP_STAGE_PAIR_ADJOINT = 4,  /* the per-pair gradients (one kernel) */
  SOAP_STAGE_FORCE_GATHER = 5,  /* per-atom force sums */
  SOAP_STAGE_GAP_FUSED = 6,     /* S, the zeta epilogue and Qbar = G Q_s in one pass (16/32-bit modes) */
  SOAP_STAGE_PAIR_PREP = 7,     /* per-pair radial factors B_k, dB_k/dr, Sec. III.A (one kernel) */
  SOAP_STAGE_CBAR = 8,          /* reserved: vbar and cbar = M c are now formed inside pair_adjoint (no launches) */
  SOAP_STAGE_PAIR_ANGULAR = 9,  /* per-pair ilexp and azimuthal factors, Sec. III.C (one kernel) */
  SOAP_STAGE_COUNT = 10
} soap_stage;
soap_status soap_profile(soap_ctx* ctx, int enable);
soap_status soap_profile_stages(soap_ctx* ctx, unsigned mask);
soap_status soap_profile_read(soap_ctx* ctx, double* ms /* host */, long long* launches /* host */);
const char* soap_stage_name(int stage);

/* Bytes of device workspace the context currently holds. */
long long soap_workspace_bytes(const soap_ctx* ctx);

/* Number of times the context's workspace has been reallocated so far (-1 for a
 * null context).  The workspace grows, by freeing and allocating, when a call
 * needs more than it holds; a HIP graph captured before a growth names freed
 * memory, so a caller that replays graphs compares this number with its value
 * at capture and captures again when it has changed.  Growth is refused with
 * SOAP_ENOTSUP while the caller's stream is being captured. */
long long soap_workspace_generation(const soap_ctx* ctx);

/*
 * Verlet skin: later neighbour builds on ctx list every pair closer than
 * r_cut + skin (0 <= skin <= r_cut; default 0).  The descriptor kernels give the
 * pairs at r >= r_cut exactly zero weight, so every result equals that of a list
 * built to r_cut (up to the order of the per-atom sums); the list stays valid
 * while no atom has moved more than skin / 2 since the build.  SOAP_EINVAL
 * outside that range.
 */
soap_status soap_set_neighbor_skin(soap_ctx* ctx, double skin);

/*
 * Pair vectors of a reused list: (dx, dy, dz)[p] = r_j + T - r_i for every listed
 * pair, from the current positions pos (n_atoms x 3, device; positions are not
 * re-wrapped into the cell, so the stored images T stay valid).  The lattice and
 * structure layout are those of the last build on ctx, which must be the build of
 * nl.  A list built with a skin is reused this way, step after step, until some
 * atom has moved more than skin / 2 since the build.  For unmoved atoms the
 * result is bitwise that of the build.  No host synchronisation.
 */
soap_status soap_update_pair_vectors(soap_ctx* ctx, const soap_nlist* nl, const double* pos, hipStream_t stream);

/* ------------------------------------------------------------------ tuning
 * Launch-shape choices that change speed, not the method.  Every setting
 * computes the same quantities and meets the same bounds; settings that change
 * the order of the GAP sums (two-pass vs fused, number of slices) agree to the
 * rounding of the operand precision; cell_split changes the order of each
 * atom's pairs in the neighbour list (not the set of pairs or their vectors),
 * hence the order of the per-atom sums; prep_block changes nothing in the
 * results.  For a fixed setting every result is bitwise reproducible.
 *   gap_fused   0: scores pass then Qbar pass; 1: one fused pass (16/32-bit
 *               modes with K <= 352; ignored otherwise)
 *   gap_slices  fused pass: target number of workgroups; the sparse set is
 *               split into slices until the grid reaches it (0: 512)
 *   prep_block  threads per block of the per-pair row kernel: 64, 128 or 256
 *   cell_split  cell-list bins of width >= r_cut / cell_split along each
 *               periodic axis (1, 2 or 3); a centre scans (2 cell_split + 1)^3
 *               bins, fewer candidate atoms for larger values.  Takes effect at
 *               the next neighbour build.
 *   gap_tile    BF16 tile shapes of the two unfused GAP passes (SOAP_MIXED_BF16
 *               and SOAP_MIXED_BF16_PS; ignored otherwise): 0: scores 128 x 128
 *               with one buffer of 128-wide K-tiles, Qbar 128 x 128 with
 *               double-buffered 64-wide K-tiles; 1: scores 128 x 128
 *               double-buffered 64-wide, Qbar 64 x 64 with 128-wide K-tiles.
 *               Same products, same summation order: bitwise the same results.
 */
typedef struct {
  int gap_fused;
  int gap_slices;
  int prep_block;
  int cell_split;
  int gap_tile;
} soap_tuning;

/* Current setting of ctx (host struct).  SOAP_EINVAL on null arguments. */
soap_status soap_get_tuning(const soap_ctx* ctx, soap_tuning* out /* host */);
/* Install a setting; SOAP_EINVAL if a field is out of range. */
soap_status soap_set_tuning(soap_ctx* ctx, const soap_tuning* t /* host */);
/* Autotuner: times gap_energy_forces (energies and forces) on the caller's
 * inputs for each candidate of each field in turn (coordinate search over
 * prep_block, gap_fused, gap_slices and gap_tile; cell_split is left as set, see
 * soap_autotune_neighbors; `repeats` timed calls per candidate after one
 * warm-up, HIP events on `stream`), keeps the fastest, installs it in ctx and
 * returns it in *chosen (host, nullable).  With a cache attached
 * (soap_set_tuning_cache) a stored setting for the same key is installed
 * instead, and a newly tuned one is stored.  Outputs go to context-owned
 * scratch; the call synchronises `stream`.  Errors as gap_energy_forces, and
 * SOAP_ENOMEM if the cache file cannot be written. */
soap_status soap_autotune(soap_ctx* ctx, const soap_nlist* nl, const int32_t* species, const double* q_sparse,
                          const double* alpha, int M, int zeta, int repeats, soap_tuning* chosen /* host */,
                          hipStream_t stream);

/* Neighbour-build autotuner: times soap_build_neighbors_async on these inputs
 * (same arguments as soap_build_neighbors) for cell_split = 1, 2, 3 (`repeats`
 * timed builds each after one warm-up, HIP events on `stream`), installs the
 * fastest in ctx and returns the whole setting in *chosen (host, nullable).  It
 * ends with one more build with the chosen setting, so that nl holds the list
 * the context's setting gives (the pair order depends on cell_split).  Returns
 * SOAP_EOVERFLOW (with *chosen untouched) if the list does not fit nl->capacity,
 * otherwise the errors of soap_build_neighbors.  Synchronises `stream`. */
soap_status soap_autotune_neighbors(soap_ctx* ctx, int n_atoms, const double* pos, const double* cells,
                                    const int32_t* pbc, const int32_t* struct_offsets, int n_structures,
                                    soap_nlist* nl, int repeats, soap_tuning* chosen /* host */,
                                    hipStream_t stream);

/* ------------------------------------------------------------- tuning cache
 * Tuned settings kept in a text file across processes.  An entry is keyed by
 * what the fastest launch shapes depend on; entries written under another
 * SOAP_TUNING_CACHE_VERSION are ignored (a library whose kernels change bumps
 * the version).  One line per entry:
 *   soap-tuning <version> <arch> <n_channels> <l_max> <K> <M> <precision>
 *     <radial_dd> <size_class> = <gap_fused> <gap_slices> <prep_block>
 *     <cell_split> <gap_tile>
 * A store replaces the entry with the same key, or appends one, and writes the
 * file anew through a temporary file and a rename.  Concurrent writers are not
 * coordinated (the last rename wins). */
#define SOAP_TUNING_CACHE_VERSION 1
typedef struct {
  int version;     /* SOAP_TUNING_CACHE_VERSION */
  int n_channels;  /* n_species * n_max */
  int l_max;
  int K;           /* descriptor length */
  int M;           /* sparse points */
  int precision;   /* soap_precision */
  int radial_dd;   /* 1: radial stage in double-double, 0: FP64 */
  int size_class;  /* floor(log2(n_atoms)) + 1; 0 for no atoms */
  char arch[32];   /* device architecture (gcnArchName up to the first ':'), NUL-terminated */
} soap_tuning_key;

/* The key of ctx's parameters for n_atoms atoms and M sparse points, on ctx's
 * device (host struct out).  SOAP_EINVAL on null arguments or negative sizes,
 * SOAP_EHIP if the device cannot be queried. */
soap_status soap_tuning_key_for(const soap_ctx* ctx, int n_atoms, int M, soap_tuning_key* out /* host */);
/* Host only (no device needed).  *found (host) = 1 and *out = the stored
 * setting if `path` holds an entry with this key (and the key's version), else
 * *found = 0; a missing file is an empty cache.  SOAP_EINVAL on null
 * arguments. */
soap_status soap_tuning_cache_lookup(const char* path, const soap_tuning_key* key, soap_tuning* out /* host */,
                                     int* found /* host */);
/* Host only.  Writes the entry (see above).  SOAP_EINVAL on null arguments or a
 * key that cannot be written on one line; SOAP_EHIP is not used; an I/O failure
 * returns SOAP_ENOMEM with the file unchanged. */
soap_status soap_tuning_cache_store(const char* path, const soap_tuning_key* key, const soap_tuning* t);
/* Attach a cache file to ctx (the path is copied; NULL detaches).  While one is
 * attached, soap_autotune first looks up the key of its inputs (soap_tuning_key_for
 * with nl->n_atoms and M): on a hit it installs the stored setting without
 * timing anything; on a miss it tunes and stores the result. */
soap_status soap_set_tuning_cache(soap_ctx* ctx, const char* path);
/* Number of soap_autotune calls on ctx answered from the cache (-1 for null). */
long long soap_tuning_cache_hits(const soap_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* SOAP_H */
