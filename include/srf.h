/*
 * srf.h -- C ABI of the short-range TreePM gravity step on MI355X (gfx950).
 *
 * The operation (Ishiyama, Nitadori & Makino, SC12, Sec. 2): given
 * positions r_i, masses m_i, the gravitational constant G, a cutoff
 * radius r_cut and a softening length eps in a periodic unit box,
 *
 *     a_i = sum_{j != i} G m_j d_ij (|d_ij|^2 + eps^2)^(-3/2) g_P3M(2 |d_ij| / r_cut),
 *
 * with d_ij the minimum image of r_j - r_i and g_P3M the cutoff function of
 * eq. (cutoff) (0 beyond r_cut).  The sum is evaluated with Barnes' modified
 * tree algorithm (Sec. 2): particles are Morton-sorted into an octree, split
 * into groups of at most n_group particles, and each group shares one
 * interaction list of particles and monopole cells, pruned by the cutoff
 * (Fig. 2) and by the opening angle theta.  The adjoint gives dL/dx and
 * dL/dm of L = sum_i w_i . a_i with the sort order, cells, groups and lists
 * held fixed.
 *
 * Calls are made in this order: srf_tree_build -> srf_make_lists ->
 * srf_short_range_force and/or srf_short_range_adjoint (and, over the same
 * tree and lists, srf_short_range_potential, or srf_short_range_quadrupole
 * after srf_short_range_force on the same output); srf_tree_refit moves a
 * tree's particles, after which srf_make_lists is called again.  srf_pm_force needs only
 * the tree; srf_kick and srf_drift need no handle.
 *
 * Memory and streams.  Unless a comment says "host", every pointer is a
 * device pointer (HIP device memory of the current device) owned by the
 * caller.  `stream` is a hipStream_t passed as void* (NULL = the null
 * stream); all device work of a call is ordered on it.  Handles (srf_tree,
 * srf_lists) own library memory and are released with srf_*_free; a handle
 * may be used only with the stream it was built on or after synchronising.
 * Handles are not thread-safe; distinct handles are.
 *
 * Errors.  Every int-returning call returns 0 (SRF_OK) or a negative
 * srf_status.  No C++ exception crosses this boundary.  srf_last_error()
 * returns a message for the most recent failure on the calling thread.
 */
#ifndef SRF_H
#define SRF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum srf_status {
    SRF_OK = 0,
    SRF_EINVAL = -1,     /* invalid argument or parameter                         */
    SRF_EDOMAIN = -2,    /* non-finite position, or mass not finite and > 0        */
    SRF_ENOMEM = -3,     /* device allocation failed                               */
    SRF_EHIP = -4,       /* a HIP runtime call failed (see srf_last_error)         */
    SRF_EMISMATCH = -5   /* tree, lists and params do not belong together          */
};

/* Opening criterion of srf_make_lists: a cell of side s is accepted as one
 * monopole iff s^2 < theta^2 d^2, d the distance from the group's box to
 * the cell's geometric centre (SRF_MAC_CENTRE, the default) or to its centre
 * of mass (SRF_MAC_COM; the pruning by r_cut stays box to box).  With
 * SRF_MAC_COM the decisions depend on the FP64 centres of mass, whose last
 * bits depend on the summation order. */
enum srf_mac {
    SRF_MAC_CENTRE = 0,
    SRF_MAC_COM = 1
};

enum srf_precision {
    SRF_FP32_REL = 0,    /* FP32 pair arithmetic on group-relative coordinates, FP64
                            positions, moments and per-particle accumulation         */
    SRF_FP64 = 1         /* all-FP64 pair arithmetic (comparison kernel)             */
};

/* Parameters.  Valid ranges (else SRF_EINVAL):
 *   G finite; 0 < r_cut < 0.25; eps > 0 and finite; 0 <= theta <= 1;
 *   1 <= n_group <= 64; 1 <= n_leaf <= n_group; precision in srf_precision;
 *   compensated in {0, 1}; mac in srf_mac. */
typedef struct {
    double G;            /* gravitational constant                                  */
    double r_cut;        /* cutoff radius, box units (box side = 1)                 */
    double eps;          /* Plummer softening length of the short-range kernel      */
    double theta;        /* opening angle; 0 accepts no cell (pure particle sums)   */
    int32_t n_group;     /* maximum particles per group                             */
    int32_t n_leaf;      /* a cell with more particles is split (down to level 21)  */
    int32_t precision;   /* enum srf_precision (force and adjoint kernels)          */
    int32_t compensated; /* 1: compensated (Kahan) FP32 partial sums over each chunk
                            of 32 list entries of the SRF_FP32_REL force kernel
                            (the chunks are added in FP64 either way); 0: plain
                            FP32.  No effect on the FP64 kernel or on the
                            adjoint.                                              */
    int32_t mac;         /* enum srf_mac: the point the opening criterion measures
                            to (srf_make_lists; must match the lists after)       */
} srf_params;

typedef struct srf_tree srf_tree;
typedef struct srf_lists srf_lists;

/* Steps a1-a5: the tree of the short-range part.  Defined by Sec. 1 (the
 * tree algorithm: particles in a hierarchy of cubic cells, each cell carrying
 * the multipole expansion of its particles, Fig. 1; the periodic box of side
 * one) and Sec. 2 (Barnes' modified algorithm: neighbouring particles form
 * groups that share one interaction list).  The paper fixes neither the key
 * nor the leaf and group rules; this call takes: wrap positions into
 * [0,1)^3, 63-bit Morton keys (21 bits per axis, x most significant in each
 * triple), stable sort by key (ties by input index), octree (a cell with
 * more than n_leaf particles is split, the root always), monopole moments
 * (mass and centre of mass, FP64), and particle groups with their tight
 * bounding boxes.
 *   n:          number of particles, 1 <= n < 2^31 - 1.
 *   x, y, z:    positions; particle i at x[i*pos_stride] (pos_stride >= 1), so
 *               an [N,3] row-major array is x = p, y = p+1, z = p+2, stride 3.
 *               Any finite value is accepted and wrapped periodically.
 *   m:          masses at m[i*m_stride]; must be finite and > 0.
 *   out:        (host) receives the new handle.
 * The inputs are copied; they may be reused once `stream` passes this call.
 * Synchronises `stream` once (to read the number of cells and groups and
 * the device's check of the inputs).  Part of the work runs on a second,
 * library-owned stream of the same device (created on first use, default
 * priority); `stream` waits for it before this call returns, so work
 * queued on `stream` afterwards sees the whole tree.
 * Errors: SRF_EINVAL, SRF_EDOMAIN (checked on the device, reported here),
 * SRF_ENOMEM, SRF_EHIP.  On error *out is NULL. */
int srf_tree_build(int64_t n, const double* x, const double* y, const double* z, int64_t pos_stride,
                   const double* m, int64_t m_stride, const srf_params* p, void* stream, srf_tree** out);

/* Tree reuse within a step (Sec. 3.1: a simulation step is one PM cycle and
 * two PP cycles; the second PP cycle may reuse the first one's tree).  The
 * particles' new positions (and, if m is not NULL, masses), in the input
 * order and number of srf_tree_build, replace the tree's; the sort order,
 * cells and groups are kept.  Positions are wrapped into [0,1)^3, and each
 * cell and group is then measured by the box of its particles instead of
 * its dyadic cube: a leaf takes its particles at their periodic images
 * nearest its dyadic centre, an inner cell the union of its children's
 * boxes, each moved by the whole number of box lengths that brings the
 * child box's centre nearest the cell's centre; a group's box holds its
 * particles' images nearest its first particle.  The monopoles are
 * recomputed from the same images (a cell whose particles lie across a
 * face of the unit box keeps them together).  srf_make_lists prunes and
 * opens on these boxes: every pair within r_cut is still found however far
 * the particles moved, but the lists grow as the boxes do, so rebuild when
 * they have moved far.  Refitting again starts from the same structure.
 * Lists built before this call are refused after it (SRF_EMISMATCH).
 *   x, y, z, pos_stride, m, m_stride: as srf_tree_build.
 * Synchronises `stream` once (the device's check of the inputs).
 * Errors: SRF_EINVAL, SRF_EDOMAIN (the tree is then unchanged), SRF_ENOMEM,
 * SRF_EHIP (the tree must then be freed). */
int srf_tree_refit(srf_tree* t, const double* x, const double* y, const double* z, int64_t pos_stride,
                   const double* m, int64_t m_stride, void* stream);

/* Step a6: per-group interaction lists.  Defined by Sec. 2 (Barnes'
 * modified algorithm: one list of cells and particles per group, built by
 * one traversal for the whole group), Fig. 2 (the short-range force needs
 * only sources within r_cut) and Sec. 1 (a well-separated cell acts through
 * its multipole; the opening test is this library's).  A cell is pruned if its periodic
 * box-to-box distance to the group's bounding box is >= r_cut, accepted as
 * one monopole if side^2 < theta^2 d^2 (d: distance from the group box to
 * the cell centre, or to its centre of mass with SRF_MAC_COM), expanded to
 * its particles if it is a leaf, and opened otherwise (the decisions are
 * made in FP64 without fused multiply-add).  For a refitted tree
 * (srf_tree_refit) each cell is its particles' box instead: the distances
 * are taken per axis to the nearest periodic image of the box centre, and
 * the side is the larger of the dyadic side and the box's longest side.
 * p must carry the n_group and n_leaf the tree was built with.  The lists
 * belong to this tree: after it is freed they are refused (SRF_EMISMATCH)
 * by every call, even with a new tree at the same address.
 * Synchronises `stream` once (to size the list buffer), twice when some
 * group's list holds more than 2048 leaves and accepted cells.
 * Errors: SRF_EINVAL, SRF_EMISMATCH, SRF_ENOMEM, SRF_EHIP. */
int srf_make_lists(const srf_tree* t, const srf_params* p, void* stream, srf_lists** out);

/* Steps a7-a8: the short-range force of Sec. 2 (the force sum over
 * particles within r_cut with the cutoff function of eq. (cutoff), written
 * out at the top of this file), evaluated over the lists of srf_make_lists.
 * Accelerations in input order, a_i = (ax[i*out_stride], ...).
 * Each group's particles interact with every list entry (particles of mass
 * m_j, cells as a particle of mass M_c at their centre of mass) through the
 * cutoff kernel; precision per p->precision.  p->r_cut, theta, n_group and
 * n_leaf must match the lists; G, eps and precision are free.
 * Fully asynchronous on `stream`.  The output may not alias the inputs.
 * Errors: SRF_EINVAL, SRF_EMISMATCH, SRF_EHIP. */
int srf_short_range_force(const srf_tree* t, const srf_lists* l, const srf_params* p,
                          double* ax, double* ay, double* az, int64_t out_stride, void* stream);

/* Step a9: not in the paper -- the derivative of the Sec. 2 force sum (as
 * evaluated by srf_short_range_force over the same lists) for a loss
 * L = sum_i w_i . a_i, with the structure fixed:
 *   dL/dx_i -> (gx, gy, gz)[i*g_stride],  dL/dm_i -> gm[i*gm_stride],
 * in input order; w_i = (wx, wy, wz)[i*w_stride].  Node sources pass their
 * gradient to member particles through M_c = sum m_k, X_c = sum m_k x_k / M_c.
 * Same parameter rules as srf_short_range_force.  Asynchronous on `stream`;
 * uses FP64 atomics, so the result is reproducible only to rounding.
 * Errors: SRF_EINVAL (also when n + number of cells exceeds 2^31 - 1),
 * SRF_EMISMATCH, SRF_ENOMEM, SRF_EHIP. */
int srf_short_range_adjoint(const srf_tree* t, const srf_lists* l, const srf_params* p,
                            const double* wx, const double* wy, const double* wz, int64_t w_stride,
                            double* gx, double* gy, double* gz, int64_t g_stride,
                            double* gm, int64_t gm_stride, void* stream);

/* Device workspace that srf_short_range_adjoint_noalloc holds on each GPU
 * it runs on, from its first call there until the process ends. */
#define SRF_NOALLOC_WORKSPACE_BYTES (128ull << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * computation, arguments and results of srf_short_range_adjoint, with every
 * workspace (the j-side and i-side partial gradients and the cells' chain
 * sums, 8 (7 n + 8 n_cells) bytes plus alignment, i.e. about 2 million
 * particles at the usual 0.15 cells per particle) taken from a static device
 * array of SRF_NOALLOC_WORKSPACE_BYTES per GPU.  It calls no hipMalloc or
 * hipFree; its first call on a device looks up that device's copy of the
 * array.  Every call on one GPU uses the same array, which keeps the last
 * call's contents (this call clears what must start at zero): calls that
 * overlap on one GPU, on other streams or threads, race.  The tree and lists
 * are built as usual (those calls allocate).  No kernel timing is recorded.
 * Errors: as srf_short_range_adjoint, and SRF_EINVAL when the tree needs
 * more workspace than the array holds (nothing is launched then). */
int srf_short_range_adjoint_noalloc(const srf_tree* t, const srf_lists* l, const srf_params* p,
                                    const double* wx, const double* wy, const double* wz, int64_t w_stride,
                                    double* gx, double* gy, double* gz, int64_t g_stride,
                                    double* gm, int64_t gm_stride, void* stream);

/* Quadrupole term of the cells (the cell expansion of Sec. 1 taken one
 * order past the monopole), ADDED to (ax, ay, az)[i*out_stride] in input
 * order: for every cell c in the list of particle i's group,
 *   G * 1/2 S_ab d_a d_b F(X_c - x_i)
 *     = G [psi S D + (psi tr(S)/2 + chi (D . S D)/2) D],   D = X_c - x_i (minimum image),
 * with S_c = sum_{k in c} m_k (x_k - X_c)(x_k - X_c)^T the cell's second
 * moments about its centre of mass, F(D) = D phi(|D|) the cutoff pair force
 * of srf_short_range_force, psi = phi'(r)/r and chi = psi'(r)/r.  Called
 * after srf_short_range_force on the same output, it gives the force with
 * quadrupole cells.  The second moments are computed by this call (FP64,
 * for the cells that occur in the lists).  Precision and parameter rules as
 * for srf_short_range_force.  Asynchronous on `stream`.  There is no
 * adjoint of this term.  Errors: SRF_EINVAL, SRF_EMISMATCH, SRF_ENOMEM,
 * SRF_EHIP. */
int srf_short_range_quadrupole(const srf_tree* t, const srf_lists* l, const srf_params* p, double* ax, double* ay,
                               double* az, int64_t out_stride, void* stream);

/* Short-range potential of the split, in input order:
 *   phi_i = -G sum_{j != i} m_j q(2 r_ij / r_cut) / (r_ij^2 + eps^2)^(1/2)   -> phi[i*out_stride]
 * over the same lists as srf_short_range_force (cells as their monopole),
 * with q the potential factor whose pair force is the cutoff of Sec. 2
 * (g = q - xi q'): q(xi) = 1 - 52/35 xi + 4/5 xi^3 - 2/5 xi^5 + 1/10 xi^6 +
 * 2/35 xi^7 - 3/140 xi^8 on [0, 1], (2 - xi)^6 (xi^2 + 4 xi + 2) / 140 on
 * [1, 2], 0 beyond.  The particle's own entry is left out (its own S2 cloud,
 * -G m_i (104/35) / r_cut, is not added).  Precision and parameter rules as
 * for srf_short_range_force; the output is written, not added.
 * Fully asynchronous on `stream`.
 * Errors: SRF_EINVAL (also when n + number of cells exceeds 2^31 - 1),
 * SRF_EMISMATCH, SRF_EHIP. */
int srf_short_range_potential(const srf_tree* t, const srf_lists* l, const srf_params* p, double* phi,
                              int64_t out_stride, void* stream);

/* Long-range (PM) half of the force split (Sec. 2 density split; PM steps
 * of Sec. 2.2, "Relay Mesh Method"), all in FP64 on a periodic n_mesh^3 mesh (points at i/n_mesh):
 * TSC assignment of the tree's particles to 27 mesh points each, 3-D FFT,
 * multiplication by -4 pi G S(k)^2 / (k^2 W(k)^2) (S the transform of the
 * S2 cloud of radius r_cut/2, W the TSC window), inverse FFT, fourth-order
 * central differences, TSC interpolation.  The accelerations are written
 * (not added) to (ax, ay, az)[i*out_stride] in input order; PP + PM is the
 * TreePM force.  Uses the sorted particles of `t`; r_cut and G need not
 * match the tree's lists, but r_cut is normally the one of the PP part.
 *   n_mesh: a power of two in [16, 1024] (memory: 40 n_mesh^3 bytes).
 * Asynchronous on `stream` (FP64 atomics: reproducible only to rounding).
 * Errors: SRF_EINVAL, SRF_ENOMEM, SRF_EHIP. */
int srf_pm_force(const srf_tree* t, double G, double r_cut, int32_t n_mesh, double* ax, double* ay, double* az,
                 int64_t out_stride, void* stream);

/* Kick and drift of the multiple-stepsize integrator (Sec. 3: a step is one
 * PM cycle and two PP cycles; the Python layer composes them):
 *   srf_kick:  v_i += dt a_i      (v, a: [i*stride] columns, device, FP64)
 *   srf_drift: x_i += dt v_i, then wrapped into [0, 1)
 * In place, asynchronous on `stream`.  Errors: SRF_EINVAL, SRF_EHIP. */
int srf_kick(int64_t n, double* vx, double* vy, double* vz, int64_t v_stride, const double* ax, const double* ay,
             const double* az, int64_t a_stride, double dt, void* stream);
int srf_drift(int64_t n, double* x, double* y, double* z, int64_t x_stride, const double* vx, const double* vy,
              const double* vz, int64_t v_stride, double dt, void* stream);

/* Release a handle (NULL is ignored).  Memory returns to the library's
 * device-memory cache; work still queued on the handle's stream stays valid. */
void srf_tree_free(srf_tree* t);
void srf_lists_free(srf_lists* l);

/* Return every cached device block to HIP (synchronises the device). */
void srf_release_cache(void);

const char* srf_strerror(int status);
const char* srf_last_error(void);

/* ---------------------------------------------------------------------
 * Inspection (all output pointers are HOST pointers; any may be NULL to
 * skip it).  These calls synchronise the handle's stream.
 * ------------------------------------------------------------------- */

/* Sizes: particles, cells, groups, deepest level. */
int srf_tree_info(const srf_tree* t, int64_t* n, int64_t* n_nodes, int64_t* n_groups, int32_t* max_level);

/* keys_sorted[n] (Morton keys in sorted order), perm[n] (input index of the
 * particle at each sorted position); cells in DFS preorder (= order of
 * (first, level)): node_level, node_prefix (top 3*level key bits),
 * node_first, node_count [n_nodes]; groups in order of first: group_first,
 * group_count [n_groups], group_lo, group_hi [n_groups*3] (tight box of the
 * wrapped positions, x,y,z per group; after srf_tree_refit, of the images
 * nearest each group's first particle).  Keys, permutation and cells are
 * those of the build; a refit keeps them. */
int srf_tree_export(const srf_tree* t, uint64_t* keys_sorted, int64_t* perm,
                    int32_t* node_level, uint64_t* node_prefix, int64_t* node_first, int64_t* node_count,
                    int64_t* group_first, int64_t* group_count, double* group_lo, double* group_hi);

/* Monopoles per cell (preorder): mass and centre of mass. */
int srf_moments_export(const srf_tree* t, double* M, double* X, double* Y, double* Z);

/* Boxes of the cells of a refitted tree (preorder, x,y,z per cell):
 * lo, hi [n_nodes*3].  SRF_EINVAL for a tree that was not refitted. */
int srf_cell_boxes_export(const srf_tree* t, double* lo, double* hi);

/* Wrapped positions and masses in sorted order [n]. */
int srf_sorted_export(const srf_tree* t, double* x, double* y, double* z, double* m);

/* List sizes: groups, particle entries, cell entries, and the interaction
 * count I = sum over groups of N_i * N_j (the paper's count, Table I). */
int srf_lists_info(const srf_lists* l, int64_t* n_groups, int64_t* n_particle_entries,
                   int64_t* n_node_entries, int64_t* interactions);

/* Lists in canonical form: per group g, particle entries
 * pidx[poff[g]..poff[g+1]) as ascending sorted indices and cell entries
 * nidx[noff[g]..noff[g+1]) as ascending preorder cell ids.  poff and noff
 * have n_groups + 1 entries. */
int srf_lists_export(const srf_lists* l, int64_t* poff, int64_t* pidx, int64_t* noff, int64_t* nidx);

/* Kernel timing (host): duration in milliseconds of the last timed
 * `srf_short_range_force` ("force") or `srf_short_range_adjoint`
 * ("adjoint") pair-kernel launch, or of the whole last `srf_pm_force`
 * ("pm"), measured with HIP events on the call's stream when timing is
 * enabled (0 disables).  The state is process-wide and not thread-safe; the
 * events are created on the device current at the first timed call, so
 * time on one device only.  srf_last_kernel_ms synchronises on the end
 * event.  Errors: SRF_EINVAL (NULL or unknown `which`, or no timed launch of
 * that kind yet), SRF_EHIP. */
int srf_set_kernel_timing(int enable);
int srf_last_kernel_ms(const char* which, double* ms);

#ifdef __cplusplus
}
#endif

#endif /* SRF_H */
