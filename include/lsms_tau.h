/*
 * liblsms_tau: the LSMS tau00 hot path on one AMD Instinct MI355X (gfx950).
 *
 * For each (site, complex energy) instance the library forms the KKR matrix
 * over the site's local interaction zone (LIZ) and returns the central block
 * of the multiple-scattering matrix,
 *     tau00 = [M^{-1}]_{00} t_0,   M = 1 - t(E) G(E),
 * which equals the central block of the Dyson-equation inverse
 * tau = [t^{-1} - g0]^{-1} (paper Sec. 2.1, eq. Dyson_equation; Sec. 2.2 for
 * the LIZ and the block-LU route that needs only the first block).
 *
 * Conventions (all entry points)
 *   - Units: Rydberg atomic units; lengths in bohr, energies in Ry.
 *   - Complex numbers are interleaved (re, im) pairs of double, i.e. the
 *     memory layout of C99 double complex / torch.complex128.
 *   - Angular index L = l*l + l + m (real spherical harmonics, no
 *     Condon-Shortley factor), kk = (lmax + 1)^2.
 *   - Matrices are column-major.
 *   - Pointers documented as "device" must point to memory of the handle's
 *     device; "host" pointers are read before the call returns.  The caller
 *     owns every buffer; the library never frees caller memory.
 *   - Every call enqueues work on `stream` (a hipStream_t, passed as void*;
 *     NULL is the default stream) and returns without synchronising.
 *     Outputs are valid after the stream has been synchronised.
 *   - Return value: 0 on success; -k when argument k (1-based) is invalid
 *     (checked on the host before anything is enqueued); LSMS_EHIP when the
 *     HIP runtime reports an error.  Per-instance status goes to info[].
 *
 * Per-instance info[i]
 *    0  success
 *   k>0, k < 2^20: an exactly zero pivot at elimination step k (1-based, in
 *       the library's elimination order: non-central columns first, the
 *       central block last, so k <= N); tau00 of the instance is NaN
 *   -1  non-finite tau00 (non-finite energy or phase shift, overflow)
 *   -2  two LIZ sites closer than 1e-8 bohr (M undefined); tau00 is NaN
 *   -3  invalid instance: empty LIZ, LIZ larger than max_liz, energy index
 *       or species out of range; tau00 is NaN and M is not written
 *   Fallback flags, ORed onto the non-negative info of the FP64 path that
 *   recomputed the instance (a negative code is reported as it is):
 *   LSMS_INFO_FP64_FALLBACK (bit 20, LSMS_PREC_FP32_IR): the refinement did
 *       not converge and the FP64 path solved the instance; info equal to the
 *       flag alone is a success, flag | k a zero pivot at step k of the FP64
 *       path.
 *   LSMS_INFO_LU_FALLBACK (bit 21, tau00_gmres): likewise for GMRES.
 *   lsms_info_pivot(info) = info & (2^20 - 1) is the zero-pivot step (0 if
 *   none) for non-negative info.
 */
#ifndef LSMS_TAU_H
#define LSMS_TAU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LSMS_EHIP (-100)

/* lsms_opts.precision */
#define LSMS_PREC_FP64 0    /* complex FP64 elimination throughout                          */
#define LSMS_PREC_FP32_IR 1 /* complex FP32 factorisation and solves (matrix cores), FP64
                               residuals and solution, iterative refinement to opts->tol;
                               an addition to the paper, whose matrices are complex FP64
                               throughout (Sec. 3.2); the refinement is the classical
                               mixed-precision scheme (Carson and Higham, SIAM J. Sci.
                               Comput. 40 (2018) A817); tau00_solve only */

/* info flag of tau00_gmres when GMRES did not reach its tolerance and the
 * instance was solved by the FP64 path (ORed onto that path's info) */
#define LSMS_INFO_LU_FALLBACK (1 << 21)
/* info flag of tau00_gmres_pc for an instance that the caller's routing sent
 * straight to the FP64 path (no GMRES step taken) */
#define LSMS_INFO_ROUTED (1 << 22)

/* learned form: parameters of the seed network and floats of activations
 * kept per sample by lsms_mlp_forward */
#define LSMS_MLP_PARAMS 399616
#define LSMS_MLP_ACT 2560

/* info flag set by LSMS_PREC_FP32_IR when the refinement did not reach tol
 * within max_refine steps (or the FP32 factorisation met an exactly zero
 * pivot) and the instance was recomputed by the FP64 path (ORed onto that
 * path's info) */
#define LSMS_INFO_FP64_FALLBACK (1 << 20)
/* mask of the zero-pivot step in a non-negative info */
#define LSMS_INFO_PIVOT_MASK ((1 << 20) - 1)

/* lsms_opts.flags */
#define LSMS_PERSISTENT 1 /* tau00_solve: one persistent fused kernel, work queue in LPT order */
#define LSMS_GRAPH 2      /* tau00_solve: capture the launches in a hipGraph on the first call with
                             a given argument set and replay it afterwards (non-null stream) */

typedef struct lsms_handle_s *lsms_handle_t;

/* One batch of (site, energy) instances with ragged LIZs.  The struct itself
 * lives in host memory; its array members are device pointers. */
typedef struct {
    int32_t lmax;        /* angular cutoff, 0..4; kk = (lmax+1)^2                      */
    int32_t n_inst;      /* number of instances (>= 0)                                 */
    int32_t n_species;   /* number of species in delta (1..8)                          */
    int32_t n_energy;    /* number of energies in energy/delta (>= 1)                  */
    int32_t max_liz;     /* upper bound on every LIZ size (1..1024); sizes workspace slots.
                            The matrix bound N = kk * max_liz (2 kk * max_liz with spin
                            canting) is at most 8192 for the batched FP64 paths, 16384
                            for build_kkr, build_kkr_spin and tau00_large, and 4096 for
                            LSMS_PREC_FP32_IR, tau00_gmres and tau_row_batched (-2
                            above)                                                      */
    int32_t reserved;
    const int64_t *liz_off;  /* device [n_inst+1]: instance i owns LIZ rows liz_off[i] ..
                                liz_off[i+1]-1 (non-decreasing, liz_off[0] = 0)       */
    const double *pos;       /* device [liz_off[n_inst]][3]: site positions relative to
                                the instance's centre; row liz_off[i] is the centre (0,0,0) */
    const int32_t *species;  /* device [liz_off[n_inst]]: species of each LIZ site,
                                in 0..n_species-1                                      */
    const double *energy;    /* device [n_energy] complex: E (Ry), Im E > 0            */
    const int32_t *e_idx;    /* device [n_inst]: energy index of each instance         */
    const double *delta;     /* device [n_species][n_energy][lmax+1] complex phase
                                shifts delta_l(E); t_l = -(1/kappa) sin(delta_l)
                                exp(i delta_l), kappa = sqrt(E) (principal branch)     */
} lsms_problem;

typedef struct {
    int32_t precision;   /* LSMS_PREC_FP64 or LSMS_PREC_FP32_IR                         */
    int32_t nb;          /* panel width of the LU, 0 = tuned value (lsms_autotune) or 128;
                            otherwise 16..128, a multiple of 16 (tau00_batched uses at
                            most 64)                                                    */
    int32_t chunk;       /* tau00_solve without LSMS_PERSISTENT: instances per pass,
                            0 = as many as fit                                          */
    int32_t flags;       /* LSMS_PERSISTENT | LSMS_GRAPH                                */
    int32_t max_refine;  /* LSMS_PREC_FP32_IR: refinement steps at most, 0 = 10; 1..100  */
    int32_t reserved;    /* must be 0                                                   */
    double tol;          /* LSMS_PREC_FP32_IR: stop once the last correction of the central
                            block is at most tol times the block (Frobenius norms), or
                            once the contraction of the last two steps (at most 1/2)
                            predicts that the next one would be (the first FP32 solve
                            counts as the step from zero, so one refinement step can
                            suffice when it predicts at most tol / 4); 0 = 1e-12;
                            otherwise 1e-15 .. 1e-3                                     */
} lsms_opts;

/* Create a handle bound to HIP device `device`: uploads the real Gaunt
 * tables (Wigner-3j closed form) for lmax = 0..4.  Returns 0 or an error. */
int lsms_create(lsms_handle_t *h, int device);

/* Release the handle's device tables. */
int lsms_destroy(lsms_handle_t h);

/* LIZ extraction (paper Sec. 2.2: each atom's KKR matrix is built over the
 * atoms of the cluster centred on it).
 *   atom_pos     device [n_atoms][3]  periodic supercell positions (bohr)
 *   atom_species device [n_atoms]
 *   box          host   [3]           orthorhombic box lengths (bohr), > 0
 *   centre       device [n_inst]      centre atom of each instance
 *   rc           device [n_inst]      cutoff radius of each instance (bohr)
 *   max_liz      rows reserved per instance (>= 1)
 * Outputs (device, caller-allocated):
 *   liz_n        [n_inst]              true LIZ size (centre included); a size
 *                                      above max_liz means the LIZ was truncated
 *   liz_off      [n_inst+1]            offsets of the compact output (sizes
 *                                      clamped to max_liz)
 *   liz_pos      [n_inst*max_liz][3]   relative positions, centre first, then by
 *                                      ascending |d|^2, ties by (dx, dy, dz)
 *   liz_species  [n_inst*max_liz]
 *   liz_atom     [n_inst*max_liz] or NULL: supercell index of each LIZ site
 * Membership: minimum-image d with dx*dx+dy*dy+dz*dz <= rc*rc (no FMA
 * contraction), each component reduced by box*rint(d/box). */
int lsms_build_liz(lsms_handle_t h, const double *atom_pos, const int32_t *atom_species, int32_t n_atoms,
                   const double *box, const int32_t *centre, const double *rc, int32_t n_inst, int32_t max_liz,
                   int32_t *liz_n, int64_t *liz_off, double *liz_pos, int32_t *liz_species, int32_t *liz_atom,
                   void *stream);

/* KKR matrix assembly (paper Sec. 2.1: M built from the single-site t and the
 * propagator between two different sites; Sec. 3.2 builds it on the CPU, the
 * paper's conclusion names building it on the GPU as the next step).
 *   M      device complex; instance i is an N_i x N_i column-major matrix at
 *          M + 2*m_off[i] doubles, N_i = kk * (liz_off[i+1] - liz_off[i]);
 *          M_ii = I_kk, M_ij = -diag(t_{s(i),l(L)}) G^{ij} with
 *          G^{ij}_{LL'} = -4 pi i kappa sum_L'' i^{l-l'+l''} C^{L''}_{LL'}
 *                          h_l''(kappa |R_ij|) Y_L''(R_ij), R_ij = R_i - R_j
 *   m_off  device [n_inst] offsets in complex elements (regions must not overlap)
 *   info   device [n_inst] out: 0 or -2 (coincident sites) */
int build_kkr(lsms_handle_t h, const lsms_problem *p, double *M, const int64_t *m_off, int32_t *info,
              void *stream);

/* tau00 from caller-built matrices (paper Sec. 2.2: block LU, first block of
 * the inverse only; Sec. 3.2: LU with partial pivoting in complex FP64).
 *   M      device complex, layout as build_kkr; overwritten by factors
 *   m_off  device [n_inst]
 *   opts   host, may be NULL (defaults)
 *   tau00  device [n_inst][kk*kk] complex out, column-major kk x kk:
 *          tau00[i][L + kk*L'] = ([M_i^{-1}]_{00} diag(t_0))_{L L'}
 *   info   device [n_inst] out
 *   work   device or NULL: with at least n_inst * LSMS_BATCHED_WORK_PER_INST
 *          bytes (the inverses of the two 64 x 64 diagonal blocks of a panel,
 *          per instance) panels may be up to 128 wide; with NULL, panels are
 *          at most 64 wide whatever opts->nb asks (work_bytes ignored).
 *          Too small a workspace returns -9.
 * Only LSMS_PREC_FP64 (the FP32 form needs the matrix unmodified and a
 * workspace: tau00_solve); another precision returns -5. */
#define LSMS_BATCHED_WORK_PER_INST (2 * 64 * 64 * 16)
int tau00_batched(lsms_handle_t h, const lsms_problem *p, double *M, const int64_t *m_off, const lsms_opts *opts,
                  double *tau00, int32_t *info, void *work, size_t work_bytes, void *stream);

/* Block row of tau through the central site and ln det M, with tau00, from
 * caller-built matrices in complex FP64.
 * tau = (t^{-1} - g0)^{-1} = M^{-1} t (paper Sec. 2.1, eq. Dyson_equation);
 * its blocks tau^{0j} over the LIZ sites j enter the Green's function of
 * eq. Green_KKR.  ln det M is the multiple-scattering term of Lloyd's formula
 * for the integrated density of states (the energy integral of eq. Density;
 * lsms_lloyd_idos turns it into that integral along the contour).
 * The elimination is tau00_batched's (pivots among the non-central rows), with
 * its upper factor kept, followed by one backward solve for the non-central
 * part of the block row.
 *   M, m_off, opts  as tau00_batched (LSMS_PREC_FP64 only, else -5)
 *   row_off  device [n_inst]: offset (complex elements) of instance i's block
 *            row in tau_row; required when tau_row is given (else -6)
 *   tau_row  device complex or NULL: instance i's kk x N_i block row,
 *            column-major with leading dimension kk:
 *            tau_row[row_off[i] + L + kk*(kk*j + L')] = tau^{0j}(L, L')
 *                = [M_i^{-1}]_{0j}(L, L') t_{s(j), l(L')}
 *            (j = 0 repeats tau00); NaN when info[i] != 0 (not written for
 *            info -3)
 *   logdet   device [n_inst] complex or NULL: ln det M_i, the imaginary
 *            part in (-pi, pi] (principal logarithm); NaN when info[i] != 0
 *   tau00, info  as tau00_batched (argument numbers 9 and 10)
 *   work     device, at least lsms_row_workspace_size bytes (-11 when NULL,
 *            -12 when too small): per instance the wide-panel blocks, the
 *            N x 16 (kk > 16: N x 32) block column of the solve and the pivots
 * Panels up to 128 wide (opts->nb or the tuned width). */
int lsms_row_workspace_size(lsms_handle_t h, const lsms_problem *p, size_t *bytes);
int tau_row_batched(lsms_handle_t h, const lsms_problem *p, double *M, const int64_t *m_off, const lsms_opts *opts,
                    const int64_t *row_off, double *tau_row, double *logdet, double *tau00, int32_t *info,
                    void *work, size_t work_bytes, void *stream);

/* Spin canting (paper Sec. 2.1 and 2.2: with canted moments every matrix
 * carries a spin index and the KKR matrix of a LIZ has rank
 * 2 N_LIZ (lmax+1)^2).  The paper gives only the rank; the library takes the
 * usual non-collinear form: site i has a unit moment direction e_i and, in
 * its own spin frame, the spin-diagonal t-matrix diag(t_up, t_dn) (t_up from
 * the phase shifts of the spin parallel to the moment); in the global frame
 *     t_i(L) = tbar_l 1 + dt_l (e_i . sigma),  tbar = (t_up + t_dn)/2,
 *     dt = (t_up - t_dn)/2,  sigma the Pauli matrices,
 * and the free propagator does not act on spin.  Row/column of (LIZ site j,
 * spin s, L): kc j + kk s + L with kc = 2 kk (s = 0: spin along global +z).
 *     M_jj = 1,  M_ij[(s,L),(s',L')] = -t_i(L)_{s s'} G^{ij}_{LL'}
 *     tau00 = [M^{-1}]_{00} t_0   (kc x kc, column-major)
 * With every moment along +z, tau00 is block-diagonal with the two plain
 * tau00 of the up and down phase shifts. */
typedef struct {
    const double *moment;    /* device [liz_off[n_inst]][3]: unit moment direction of each LIZ
                                site, per LIZ row like lsms_problem.pos (lsms_liz_moments)   */
    const double *delta_dn;  /* device [n_species][n_energy][lmax+1] complex: phase shifts of
                                the spin antiparallel to the site's moment (lsms_problem.delta
                                then holds the parallel spin)                               */
} lsms_spin;

/* liz_moment[r] = atom_moment[liz_atom[r]] (3 doubles per row) for the rows of
 * lsms_build_liz (liz_atom its optional output); NaN for an atom index
 * outside [0, n_atoms).  Errors: -2 n_rows < 0, -3/-4/-6 null, -5 n_atoms < 1. */
int lsms_liz_moments(lsms_handle_t h, int64_t n_rows, const int32_t *liz_atom, const double *atom_moment,
                     int32_t n_atoms, double *liz_moment, void *stream);

/* build_kkr with spin canting: instance i is a kc N_LIZ square at M + 2*m_off[i]
 * doubles (N_i = 2 kk N_LIZ,i <= 16384).  Arguments as build_kkr, spin third
 * (-3 when NULL or, for a nonempty batch, with a NULL member). */
int build_kkr_spin(lsms_handle_t h, const lsms_problem *p, const lsms_spin *spin, double *M, const int64_t *m_off,
                   int32_t *info, void *stream);

/* tau00_batched with spin canting: tau00 [n_inst][kc*kc] complex, column-major
 * per instance, tau00[i][a + kc*b] = tau00_i(a, b), a = kk s + L.  FP64 only
 * (another precision or invalid opts: -6); work as tau00_batched (-10 when
 * too small). */
int tau00_spin_batched(lsms_handle_t h, const lsms_problem *p, const lsms_spin *spin, double *M,
                       const int64_t *m_off, const lsms_opts *opts, double *tau00, int32_t *info, void *work,
                       size_t work_bytes, void *stream);

/* Workspace and fused build + solve (as lsms_workspace_size / tau00_solve:
 * chunked passes or LSMS_PERSISTENT) with spin canting; FP64 only, no
 * LSMS_GRAPH (-4 otherwise).  A slot holds one kc N_LIZ square matrix
 * (298 MB at rank 4320, 729 MB at rank 6750).  tau00_spin_solve returns -8
 * when work_bytes is too small. */
int lsms_spin_workspace_size(lsms_handle_t h, const lsms_problem *p, const lsms_spin *spin, const lsms_opts *opts,
                             int32_t chunk, size_t *bytes);
int tau00_spin_solve(lsms_handle_t h, const lsms_problem *p, const lsms_spin *spin, const lsms_opts *opts,
                     double *tau00, int32_t *info, void *work, size_t work_bytes, void *stream);

/* One instance across the whole GPU (paper Sec. 5: offloading the inverse of
 * the whole KKR matrix; Sec. 4.1: ranks 6225 to 12450).  tau00 of a single
 * caller-built matrix with every compute unit taking part: per panel of 64
 * columns ceil(rows / 128) workgroups factorise the panel together (partial
 * pivoting among the non-central rows, as tau00_batched; each workgroup
 * holds 128 of the panel's rows in LDS, one grid barrier per column for the
 * pivot choice; the workgroups of a panel are at most 128, one per compute
 * unit, and every barrier wait gives up after a bounded number of polls),
 * then one workgroup per 64-column strip applies the interchanges and forms
 * U12, and workgroups of 128 to 2048 rows of a strip apply the MFMA update;
 * the next panel is factorised while the rest of the update runs (one panel
 * of look-ahead, on a second stream of the handle, joined back to `stream`
 * before the call's last kernel).
 *   p        n_inst = 1, the instance's LIZ exactly max_liz sites (info -3
 *            otherwise); N = kk * max_liz (2 kk * max_liz with spin) <= 16384
 *   spin     NULL, or spin canting as tau00_spin_batched
 *   M        device complex N x N column-major (build_kkr / build_kkr_spin with
 *            m_off = 0); overwritten
 *   opts     FP64 only, nb 0 or 64, no flags (-5 otherwise)
 *   tau00, info  device, one instance (as tau00_batched / tau00_spin_batched);
 *            info -4 when a barrier wait gave up (lsms_large_set_spin_limit)
 *   work     device, lsms_large_workspace_size bytes (pivots, two 64 x 64
 *            blocks; -8 when NULL, -9 when too small)
 * Returns -10 when the device cannot hold all ceil(N / 128) workgroups of
 * the first panel at once (queried with the occupancy API at lsms_create;
 * a barrier needs them all resident).
 * Calls on one handle must not overlap in time (they share the second stream
 * and its events). */
int lsms_large_workspace_size(lsms_handle_t h, const lsms_problem *p, const lsms_spin *spin, size_t *bytes);
/* Polls of one grid-barrier wait of tau00_large's panel kernel before it
 * gives up (0: the default, several seconds).  A wait that gives up makes
 * every workgroup of that panel and every later panel leave at once, and the
 * instance reports info -4 with tau00 NaN; all kernels still end normally.
 * Errors: -2 polls < 0. */
int lsms_large_set_spin_limit(lsms_handle_t h, int64_t polls);
int tau00_large(lsms_handle_t h, const lsms_problem *p, const lsms_spin *spin, double *M, const lsms_opts *opts,
                double *tau00, int32_t *info, void *work, size_t work_bytes, void *stream);

/* Energy integration along the contour (paper Sec. 2.1, eq. Density: the
 * density of states and the charge are energy integrals, taken by quadrature
 * on a complex contour).  A batch is laid out [site][energy], instance
 * s * n_energy + k, the energies in contour order.
 *   weights  device [n_energy] complex quadrature weights of the contour
 *   values   device [n_sites][n_energy][m] complex (e.g. tau00 with m = kk*kk)
 *   out      device [n_sites][m] complex: out[s][c] = sum_k weights[k] values[s][k][c]
 * Errors: -2 n_sites < 0, -3 n_energy < 1, -4 m < 0, -5..-7 null pointers. */
int lsms_contour_sum(lsms_handle_t h, int32_t n_sites, int32_t n_energy, int32_t m, const double *weights,
                     const double *values, double *out, void *stream);

/* Lloyd's formula along the contour: from ln det M at the contour's nodes
 * (logdet device [n_sites][n_energy] complex, in contour order, as returned
 * by tau_row_batched), the multiple-scattering integrated density of states
 * relative to the first node, idos device [n_sites][n_energy] double:
 *     idos[s][k] = -(phi_k - phi_0) / pi,
 * phi the phase of det M followed continuously from node to node, each step
 * being the difference of the principal phases reduced to [-pi, pi] (the
 * phase must move by less than pi between neighbouring nodes).
 * Errors: -2 n_sites < 0, -3 n_energy < 1, -4/-5 null pointers. */
int lsms_lloyd_idos(lsms_handle_t h, int32_t n_sites, int32_t n_energy, const double *logdet, double *idos,
                    void *stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): tau00_batched
 * without the workspace argument and without any allocation.  The wide-panel
 * blocks live in a scratch array of the library, 32 MiB per device (room for
 * 256 instances), held from lsms_create until the process ends; the batch is
 * processed in stream-ordered passes of at most 256 instances, so n_inst has
 * no upper limit beyond tau00_batched's own checks (kk * max_liz <= 8192,
 * -2 above).  Panels up to 128 wide (opts->nb, or the tuned width).  The call
 * enqueues kernel launches only (no hipMalloc, hipFree, memset or copy).
 * Every call on one device shares that device's array: calls that overlap in
 * time on one device (different streams, or threads) race and give undefined
 * results; calls ordered on one stream do not.  Arguments, outputs and errors
 * as tau00_batched (LSMS_PREC_FP64 only, else -5). */
int tau00_batched_noalloc(lsms_handle_t h, const lsms_problem *p, double *M, const int64_t *m_off,
                          const lsms_opts *opts, double *tau00, int32_t *info, void *stream);

/* Workspace of tau00_solve.  Without LSMS_PERSISTENT: `chunk` instances per
 * pass, one slot per instance.  With LSMS_PERSISTENT (chunk ignored): one
 * 256-byte-aligned slot per resident workgroup of the persistent kernel (one
 * per compute unit), plus a work counter and the instance order (4 bytes per
 * instance).  A slot holds the FP64 matrix, n^2 * 16 bytes for
 * n = kk*max_liz, and the inverses of the two diagonal blocks of a panel
 * wider than 64 (2 * 64 * 64 * 16 bytes); with LSMS_PREC_FP32_IR also the
 * matrix's FP32 copy (n^2 * 8), the FP32 and FP64 right-hand sides
 * (n * kp * 24, kp = 16 or 32) and the pivots (n * 4); each part 256-byte
 * aligned. */
int lsms_workspace_size(lsms_handle_t h, const lsms_problem *p, const lsms_opts *opts, int32_t chunk,
                        size_t *bytes);

/* Fused LIZ-to-tau00 solve (paper Sec. 2.2 per LIZ, Sec. 5: M built on the
 * GPU): M never leaves the device workspace.
 * Without LSMS_PERSISTENT the instances are processed in passes of
 * floor(work_bytes / slot) (or opts->chunk) instances, each pass a build
 * launch and an elimination launch.  With LSMS_PERSISTENT, one launch of
 * resident workgroups takes instances from a device counter in order of
 * decreasing LIZ size (longest first), builds each M in the workgroup's own
 * slot and eliminates it; ragged batches need no padding.  With LSMS_GRAPH
 * the launches are captured once per argument set into a hipGraph kept by
 * the handle and replayed (if `stream` is already capturing, the launches
 * are simply recorded into the caller's capture).  Arguments as
 * tau00_batched; work is a device buffer of lsms_workspace_size bytes. */
int tau00_solve(lsms_handle_t h, const lsms_problem *p, const lsms_opts *opts, double *tau00, int32_t *info,
                void *work, size_t work_bytes, void *stream);

/* Autotuner: times tau00_solve (with opts->flags, without LSMS_GRAPH) on the
 * problem for panel widths nb = 32, 64, 96, 128, each after one warm-up call
 * and as the median of three timed calls, stores the fastest as the handle's
 * panel width for matrices of this problem's size bucket (kk*max_liz rounded
 * up to a multiple of 128) and precision (opts->precision; tuned widths of
 * the FP64 path and of the precision form are kept apart), returns it in
 * *best_nb and the four median timings (ms, in the order above) in ms_out[4]
 * (host, or NULL).  Synchronises the stream. */
int lsms_autotune(lsms_handle_t h, const lsms_problem *p, const lsms_opts *opts, double *tau00, int32_t *info,
                  void *work, size_t work_bytes, void *stream, int32_t *best_nb, double *ms_out);

/* Sets (get: reads, 0 = not tuned) the handle's panel width for matrices of
 * size n (1..4096, the bucket of lsms_autotune) in the given precision
 * (LSMS_PREC_FP64 or LSMS_PREC_FP32_IR), e.g. from a cached tuning result.
 * nb: 16..128, a multiple of 16. */
int lsms_set_tuned_nb(lsms_handle_t h, int32_t n, int32_t precision, int32_t nb);
int lsms_get_tuned_nb(lsms_handle_t h, int32_t n, int32_t precision, int32_t *nb);

/* The handle's tuned panel widths to a file (host path) and back: a JSON
 * array with one object {"n_max": n, "precision": p, "nb": w} per line, n the
 * upper end of the size bucket.  lsms_autotune_load sets every entry of that
 * form it finds (lines of any other form are skipped) and reports their
 * number in *n_loaded (or NULL).  Return -2 when the file cannot be opened
 * or written. */
int lsms_autotune_save(lsms_handle_t h, const char *path);
int lsms_autotune_load(lsms_handle_t h, const char *path, int32_t *n_loaded);

/* ---------------------------------------------------------------------------
 * Learned form.  The paper solves every instance directly (Sec. 3.2); this
 * form adds a small network that maps an instance's local environment and
 * energy to an approximation of [M^{-1}]_{00}, which seeds an iterative block
 * GMRES solve of the same system; the direct FP64 path is the fallback.
 *
 * Network: 18 -> 256 -> 256 -> 256 -> 1024, SiLU after the hidden layers,
 * linear output.  Parameters: one flat float array of LSMS_MLP_PARAMS
 * entries [W1 b1 W2 b2 W3 b3 W4 b4], W_l row-major [out][in]; the products
 * use a bf16 copy of it (uint16 bit patterns, same layout) and round the
 * layer inputs to bf16, with FP32 accumulation.  Outputs per sample: 512
 * floats for tau00 and 512 for [M^{-1}]_{00} (kk = 16, column-major,
 * interleaved re/im), both normalised (see lsms_mlp_seed).
 * -------------------------------------------------------------------------*/

/* Features of each instance (device [n_inst][18] floats): the centre's
 * species one-hot (species 0 and 1), for the first seven fcc neighbour
 * shells (ideal radii a_lat*sqrt(k/2)) the fraction of the shell's sites of
 * species 0 and 1 (each LIZ site counted in the shell nearest in radius;
 * sites nearest to the eighth shell are not counted), Re E, Im E.  The
 * problem's LIZ arrays as for tau00_solve (lsms_build_liz output). */
int lsms_mlp_features(lsms_handle_t h, const lsms_problem *p, double a_lat, float *feat, void *stream);

/* w_bf16 (device, LSMS_MLP_PARAMS uint16) := bf16(params), round to nearest
 * even. */
int lsms_mlp_cast(lsms_handle_t h, const float *params, uint16_t *w_bf16, void *stream);

/* Forward pass over n samples: feat device [n][18]; act device [n][LSMS_MLP_ACT]
 * (pre-activations and activations kept for the backward pass, outputs in
 * the last 1024 floats of each row); out device [n][1024] or NULL. */
int lsms_mlp_forward(lsms_handle_t h, const float *params, const uint16_t *w_bf16, const float *feat, int32_t n,
                     float *out, float *act, void *stream);

/* Backward pass: grad (device, LSMS_MLP_PARAMS floats, overwritten) of
 * sum(dout * out) for the forward that filled act; the bf16 rounding of the
 * forward is taken as the identity.  work: device [n][1280] floats. */
int lsms_mlp_backward(lsms_handle_t h, const uint16_t *w_bf16, const float *feat, const float *act,
                      const float *dout, int32_t n, float *grad, float *work, void *stream);

/* Mean squared error over `count` floats: *loss (device) = mean (out-target)^2,
 * dout = its gradient 2 (out - target) / count. */
int lsms_mlp_mse(lsms_handle_t h, const float *out, const float *target, int64_t count, float *dout, float *loss,
                 void *stream);

/* AdamW step `step` (1-based) on the FP32 parameters (moments m, v device
 * floats, zero before step 1), refreshing w_bf16:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * w -= lr (m/(1-b1^step) / (sqrt(v/(1-b2^step)) + eps) + weight_decay w). */
int lsms_mlp_adamw(lsms_handle_t h, float *params, uint16_t *w_bf16, float *m, float *v, const float *grad, float lr,
                   float beta1, float beta2, float eps, float weight_decay, int32_t step, void *stream);

/* Seeds for tau00_gmres from network outputs out [n][1024]:
 * seed[i] (device [n][256] complex, column-major 16 x 16) =
 * out[i][512 + q] * scale[512 + q] + shift[512 + q] for the 512 floats q
 * (scale, shift device [1024] floats, the training normalisation). */
int lsms_mlp_seed(lsms_handle_t h, const float *out, const float *scale, const float *shift, int32_t n,
                  double *seed, void *stream);

/* Training targets of each instance (device [n_inst][1024] floats) from
 * tau00 (device [n_inst][256] complex, e.g. tau00_solve's output):
 * [tau00 | D], D(L, L') = tau00(L, L') / t0_{l(L')} = [M^{-1}]_{00}(L, L')
 * (0 where t0 vanishes), interleaved re/im, column-major 16 x 16 each.  With
 * scale and shift (device [1024] floats, both or neither) the targets are
 * normalised: (x - shift) / scale.  lmax = 3. */
int lsms_mlp_targets(lsms_handle_t h, const lsms_problem *p, const double *tau00, const float *scale,
                     const float *shift, float *target, void *stream);

/* Normalisation of targets [n][1024]: shift = column mean, scale = column
 * standard deviation (1 where it vanishes). */
int lsms_mlp_norm_stats(lsms_handle_t h, const float *target, int32_t n, float *scale, float *shift, void *stream);

/* Workspace of tau00_gmres: one slot per resident workgroup (the matrix, the
 * two 64 x 64 blocks of the fallback, the solution, the residual, restart+1
 * Krylov blocks of n x 16 complex, the block Hessenberg matrix) plus the work
 * counter and the instance order.  lmax must be 3 (-2 otherwise);
 * 1 <= restart <= 8 (-3). */
int lsms_gmres_workspace_size(lsms_handle_t h, const lsms_problem *p, int32_t restart, size_t *bytes);

/* tau00 by block GMRES (lmax = 3): for each instance the fused kernel builds
 * M as tau00_solve does and solves A Y = E_c (A = M^T, E_c the 16 unit columns
 * of the central block) with all 16 columns as one block: restarted block
 * GMRES(restart) from Y_c = seed^T in the central rows (or zero if seed is
 * NULL) followed by one Jacobi step on the other rows, until
 * ||E_c - A Y||_F <= tol ||E_c||_F or max_cycles restarts; then
 * tau00 = Y_c^T diag(t_0).  An instance that does not converge is solved by
 * the FP64 path (info = LSMS_INFO_LU_FALLBACK).  steps: device [n_inst], block
 * Arnoldi steps (one product with M each) taken.  seed: device [n_inst][256]
 * complex approximation of [M^{-1}]_{00} (lsms_mlp_seed) or NULL. */
int tau00_gmres(lsms_handle_t h, const lsms_problem *p, const double *seed, int32_t restart, int32_t max_cycles,
                double tol, double *tau00, int32_t *info, int32_t *steps, void *work, size_t work_bytes,
                void *stream);

/* tau00_gmres with a block-diagonal right preconditioner and per-instance
 * routing (both optional, NULL for none; the other arguments as tau00_gmres,
 * their error numbers shifted by three):
 *   precond      device [n_blocks][256] complex, column-major 16 x 16 blocks
 *                D_b approximating a site's diagonal block of M^{-1} (the
 *                network's [M^{-1}]_{00} of the instance centred on that site,
 *                lsms_mlp_seed); GMRES then solves A P^{-1} Z = E_c,
 *                Y = P^{-1} Z, with P^{-1} block-diagonal over the LIZ sites,
 *                the block of site j being D_{row[j]}^T (A = M^T)
 *   precond_row  device [liz_off[n_inst]]: the block of every LIZ row, < 0 for
 *                the identity (lsms_site_blocks); required with precond (-5)
 *   route        device [n_inst] int8 or NULL: nonzero sends the instance
 *                straight to the FP64 path (info |= LSMS_INFO_ROUTED, steps 0)
 * The stopping test is on the true residual ||E_c - A Y||_F. */
int tau00_gmres_pc(lsms_handle_t h, const lsms_problem *p, const double *seed, const double *precond,
                   const int32_t *precond_row, const int8_t *route, int32_t restart, int32_t max_cycles, double tol,
                   double *tau00, int32_t *info, int32_t *steps, void *work, size_t work_bytes, void *stream);

/* Preconditioner block of every LIZ row for tau00_gmres_pc when the batch
 * itself holds the blocks: precond_row[r] = the instance i of the batch with
 * centre[i] = liz_atom[r] and the energy of the row's own instance (-1 when
 * the batch has no such instance).  liz_atom: device [liz_off[n_inst]]
 * (lsms_build_liz), centre: device [n_inst] supercell indices of the
 * instances' centres, work: device n_atoms * n_energy ints.
 * Errors: -3/-4/-6/-7 null pointers, -5 n_atoms < 1. */
int lsms_site_blocks(lsms_handle_t h, const lsms_problem *p, const int32_t *liz_atom, const int32_t *centre,
                     int32_t n_atoms, int32_t *precond_row, int32_t *work, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LSMS_TAU_H */
