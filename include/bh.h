/*
 * bh.h -- C ABI of the MI355X (gfx950) Barnes-Hut tree-code library.
 *
 * The library computes one gravitational force evaluation and one
 * leapfrog step of a particle system on one GPU, following the tree-code of
 * Bedorf et al., "24.77 Pflops on a Gravitational Tree-Code to Simulate the
 * Milky Way Galaxy with 18600 GPUs" (SC14):
 *
 *   tree_build     bounding box, space-filling-curve keys and key sort
 *                  (Sec. III.B.1; Table II "Sorting SFC"), octree
 *                  construction with at most 16 particles per leaf (Sec. I.A;
 *                  Table II "Tree-construction"), target groups, and the
 *                  multipole moments of every cell (Sec. I.A; Table II
 *                  "Tree-properties")
 *   tree_force     the group-wise tree walk with opening angle theta, fused
 *                  with the force evaluation of Sec. VI.A Eq. (1)-(2)
 *                  (Sec. III.A; Table II "Compute gravity")
 *   leapfrog_step  one second-order kick-drift-kick leapfrog step with a full
 *                  tree rebuild (Sec. III.B.2)
 *
 * Conventions for every entry point:
 *   - G = 1.  Positions are [N][3] row-major FP32, masses [N] FP32 (> 0).
 *   - "device" pointers are HIP device allocations on the context's device;
 *     "host" pointers are ordinary host memory.
 *   - Work is enqueued on the caller's HIP stream `s` (0 = the null stream)
 *     and runs asynchronously unless the entry point says it synchronises.
 *     A context must be used from one host thread and one stream at a time;
 *     the library takes no locks.
 *   - Every call returns BH_OK (0) or a negative bh_status; nothing aborts
 *     or throws across the ABI.  bh_last_error() describes the last failure.
 *   - Conditions found on the device (a non-finite position or a
 *     non-positive mass at build time) are latched in a device status word
 *     and reported by the next synchronising call (bh_sync, bh_stats_get,
 *     bh_export, bh_export_keys, bh_export_tree, bh_get_state).
 */
#ifndef BH_H
#define BH_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum bh_status {
    BH_OK = 0,
    BH_EINVAL = -1,      /* an argument is out of range (n <= 0, theta outside
                            (0, 1], eps < 0 or not finite, dt not finite,
                            null pointer, unknown export id) */
    BH_ECAPACITY = -2,   /* n > n_max of the context, or an export buffer is
                            too small */
    BH_ENOMEM = -3,      /* device allocation failed in bh_create */
    BH_EHIP = -4,        /* a HIP runtime call failed */
    BH_ENONFINITE = -5,  /* device status: non-finite position or velocity */
    BH_ESTATE = -6,      /* call out of order (force or step before a build) */
    BH_EMASS = -7        /* device status: a mass is <= 0 or not finite */
} bh_status;

/* Tree parameters, fixed for the lifetime of a context. */
typedef struct bh_params {
    int32_t nleaf;    /* a cell holding more than nleaf particles is split
                         (Sec. I.A uses 16); 1..64 */
    int32_t ncrit;    /* target groups hold at most ncrit particles; 1..64 */
    int32_t far_fp16; /* 1: particle-cell (far-field) terms in packed FP16 with
                         FP32 accumulation, each (group, cell) pair rescaled by
                         powers of two so FP16 values are of order one; pairs too
                         close for that range, and all particle-particle terms,
                         stay FP32.  Same interaction lists as 0 (FP32). */
    int32_t pos_fp64; /* 1: keep an FP64 master copy of the positions; the
                         leapfrog drift is done in FP64 and the tree is built
                         from its FP32 rounding.  0: FP32 positions. */
    int32_t adjoint;  /* 1: allocate the buffers of tree_force_vjp: FP64 cell and
                         particle adjoints, one copy per XCD (8): 640 bytes per
                         cell of capacity + 276 bytes per particle, and 168 MB
                         for 32 further copies of the first 65536 cells' */
    int32_t curve;    /* space-filling curve of the keys: 0 Morton, 1 Peano-Hilbert
                         (the paper's, Sec. III.B.1).  Every octree cell is one key
                         range under both, so the cells are the same; only their
                         order and the particle order inside them differ. */
    int32_t pair_groups; /* 0: off (the target groups above).  2..64: two
                         consecutive groups 2k, 2k + 1 whose cells are siblings
                         and that hold at most pair_groups particles together
                         are walked as one target set, against the box of their
                         union (Sec. III.A walks a group of targets at a time;
                         the paper does not fix how targets are grouped).  Fewer
                         walks, more interactions per target: the forces are the
                         same method's, with more particle-particle terms. */
    int32_t reserved;
} bh_params;

typedef struct bh_ctx bh_ctx;

/* Create a context on the current HIP device with room for up to n_max
 * particles.  The context owns every buffer the path needs (sorted particle
 * state, keys, cells, moments, groups); they are allocated here, once.
 * p == NULL selects nleaf = 16, ncrit = 64.  On success *out is set. */
int bh_create(bh_ctx **out, int64_t n_max, const bh_params *p);

/* Free the context and all its device memory (synchronises the device). */
int bh_destroy(bh_ctx *ctx);

/* Build the tree for n particles (Sec. III.B.1, Sec. I.A).
 *   pos   device, [n][3] FP32, caller order
 *   mass  device, [n] FP32, caller order, every mass > 0
 * The particle state becomes (pos, velocity 0, mass).  The inputs are read
 * by work enqueued on s; the caller may reuse them once s has passed that
 * point.  Errors: BH_EINVAL (n <= 0, null pointer), BH_ECAPACITY
 * (n > n_max); non-finite positions / bad masses are latched. */
int tree_build(bh_ctx *ctx, const float *pos, const float *mass, int64_t n, hipStream_t s);

/* Set positions, velocities and masses (device, caller order; vel may be
 * NULL for zero velocities) and build the tree for them.  Same errors as
 * tree_build. */
int bh_set_state(bh_ctx *ctx, const float *pos, const float *vel, const float *mass, int64_t n,
                 hipStream_t s);

/* Forces on every particle from the last built tree (Sec. III.A, Sec. VI.A
 * Eq. (1)-(2) with Plummer softening eps).
 *   theta  opening angle, 0 < theta <= 1
 *   eps    softening length >= 0
 *   acc    device, [n][3] FP32, caller order (may be NULL)
 *   pot    device, [n] FP32, caller order (may be NULL); the self pair is
 *          excluded from the potential
 * The outputs are valid once s has passed this work.  Errors: BH_EINVAL,
 * BH_ESTATE (no tree built). */
int tree_force(bh_ctx *ctx, float theta, float eps, float *acc, float *pot, hipStream_t s);

/* Direct summation in FP64 at chosen particles over all n particles of the
 * current state: the theta -> 0 limit of the tree force (Sec. I.A), the
 * reference the error of tree_force is stated against.  Positions are the
 * FP32 values the tree is built from; the self pair is skipped, and so is a
 * zero-separation pair when eps = 0.
 *   targets  device, [nt] caller indices in [0, n)
 *   acc      device, [nt][3] FP64, overwritten
 *   pot      device, [nt] FP64, overwritten
 * Spans of sources are combined with FP64 atomics (last-bit differences
 * between runs are possible).  Errors: BH_EINVAL (bad eps, nt < 0, null
 * pointer; an index outside [0, n) leaves its outputs 0 and is latched as
 * BH_EINVAL for the next synchronising call), BH_ESTATE (no tree). */
int tree_direct(bh_ctx *ctx, const int64_t *targets, int64_t nt, float eps, double *acc,
                double *pot, hipStream_t s);

/* One kick-drift-kick step (Sec. III.B.2): v += a dt/2; x += v dt; rebuild
 * the tree; a = force(x); v += a dt/2.  The force at the current state is
 * computed first when the last call did not leave one for (theta, eps).
 * Errors: BH_EINVAL (dt not finite, theta/eps out of range), BH_ESTATE. */
int leapfrog_step(bh_ctx *ctx, float dt, float theta, float eps, hipStream_t s);

/* Adjoint of tree_force with the walk's decisions held fixed (the opening
 * decisions, tree topology and group boxes are piecewise constant and have
 * zero derivative): for the cotangent u of the accelerations,
 *   g_pos  += coef * u^T d(acc)/d(pos)     (device, [n][3], caller order)
 *   g_mass += coef * u^T d(acc)/d(mass)    (device, [n], caller order)
 * either output may be NULL.  The accelerations are those of Sec. VI.A
 * Eq. (2) over the lists of a walk of the current tree with (theta, eps);
 * cells enter through their moments (Sec. I.A, Eq. (1)), whose adjoint is
 * applied to every particle of every cell.  u is device [n][3] caller order.
 * Source terms are reduced with FP64 atomics, so results may differ in the
 * last bits between runs.  Errors: BH_EINVAL (bad theta/eps, null u, context
 * without adjoint = 1), BH_ESTATE (no tree). */
int tree_force_vjp(bh_ctx *ctx, float theta, float eps, const float *u, float coef,
                   float *g_pos, float *g_mass, hipStream_t s);

/* Transpose of the drift x += dt v of the kick-drift-kick leapfrog
 * (Sec. III.B.2) for the adjoint sweep: gv += dt * gx (device, [n][3],
 * caller order).  Errors: BH_EINVAL (null pointer, dt not finite),
 * BH_ESTATE (no state). */
int leapfrog_vjp_drift(bh_ctx *ctx, float dt, const float *gx, float *gv, hipStream_t s);

/* Flags of leapfrog_vjp_segment. */
enum {
    BH_SEG_FIRST = 1, /* the segment starts at the trajectory's initial state:
                         its first kick transpose takes dt/2 */
    BH_SEG_LAST = 2   /* the segment ends at the trajectory's final state: the
                         last step's closing half kick is transposed first */
};

/* Reverse sweep of k kick-drift-kick leapfrog steps (Sec. III.B.2) from a
 * checkpoint, with the walk's decisions held fixed as in tree_force_vjp.
 *   snap      device, a snapshot of the state x_s at the segment's first step
 *             (bh_save_state of this context with n particles); read only
 *   k         steps in the segment, >= 1
 *   flags     BH_SEG_FIRST / BH_SEG_LAST (0 for an interior segment)
 *   dt, theta, eps   those of the forward steps (leapfrog_step)
 *   gx, gv    device, [n][3] caller order: cotangents of (x, v) after the
 *             segment's k steps; read only
 *   gx0, gv0  device, [n][3]: overwritten with the cotangents of (x, v) at
 *             the segment's start; they may be the same buffers as gx, gv
 *   gm        device, [n]: the masses' gradient is ADDED to it (may be NULL)
 * The call restores snap, recomputes the states inside the segment with
 * leapfrog_step (so trees and decisions are bit-identical to the forward
 * run's), then walks back step by step: the drift transpose gv += dt gx and
 * one force adjoint per position, gx += c J^T gv, gm += c Jm^T gv, where the
 * two half kicks meeting at an interior position share c = dt, and c = dt/2
 * at the trajectory's ends (BH_SEG_FIRST, BH_SEG_LAST).  Calling it once per
 * checkpoint segment, last segment first, gives the K-step gradient.
 * On return the context holds a state of the segment (not the caller's
 * latest).  The k - 1 recomputed states are kept in a context-owned device
 * buffer of (k - 1) * bh_state_bytes() bytes, allocated on first need and
 * grown when a call needs more.  Errors: BH_EINVAL (null pointer, k < 1,
 * unknown flags, dt / theta / eps out of range, context without
 * adjoint = 1), BH_ECAPACITY (n > n_max), BH_ENOMEM (segment buffer). */
int leapfrog_vjp_segment(bh_ctx *ctx, const void *snap, int64_t n, int32_t k, int32_t flags,
                         float dt, float theta, float eps, const float *gx, const float *gv,
                         float *gx0, float *gv0, float *gm, hipStream_t s);

/* Bytes of a state snapshot for the current n (0 if nothing built). */
int64_t bh_state_bytes(const bh_ctx *ctx);

/* Snapshot the particle state exactly as held (sorted order, caller
 * indices, FP64 positions if kept) into device memory dst of
 * bh_state_bytes() bytes.  Loading it later reproduces the same tree, the
 * same walk and so bit-identical steps; this is how the adjoint sweep
 * replays a checkpointed trajectory, and it serves as a restart point. */
int bh_save_state(bh_ctx *ctx, void *dst, hipStream_t s);

/* Restore a snapshot of n particles (device memory) and rebuild the tree. */
int bh_load_state(bh_ctx *ctx, const void *src, int64_t n, hipStream_t s);

/* Polar grid of the surface-density observable. */
typedef struct bh_cic_grid {
    float r_min, r_max;   /* radial range, 0 < r_min < r_max; particles outside
                             it are dropped (the inner cut bounds d(phi)/dx) */
    int32_t n_r, n_phi;   /* cells; n_r * n_phi <= 65536 */
} bh_cic_grid;

/* Face-on surface density of the selected particles (sel: device [n] bytes,
 * nonzero = selected, NULL = all) on the polar grid, cloud-in-cell in
 * (R, phi) with phi periodic: cell centres R_i = r_min + (i + 1/2) dR,
 * phi_j = (j + 1/2) dphi; mass / cell area.  pos device [n][3], mass [n],
 * density device [n_r][n_phi]. */
int bh_cic_density(bh_ctx *ctx, const float *pos, const float *mass, const uint8_t *sel,
                   int64_t n, const bh_cic_grid *grid, float *density, hipStream_t s);

/* Adjoint of bh_cic_density: g_pos += (d density/d pos)^T g_density,
 * g_mass += (d density/d mass)^T g_density (device, caller order; either may
 * be NULL). */
int bh_cic_density_vjp(bh_ctx *ctx, const float *pos, const float *mass, const uint8_t *sel,
                       int64_t n, const bh_cic_grid *grid, const float *g_density,
                       float *g_pos, float *g_mass, hipStream_t s);

/* Copy the particle state out in caller order (device pointers, [n][3];
 * either may be NULL).  Synchronises s and reports latched device status. */
int bh_get_state(bh_ctx *ctx, float *pos, float *vel, hipStream_t s);

/* Conserved quantities of the current state in FP64 (host out[9]):
 *   out[0]     total mass
 *   out[1]     kinetic energy  1/2 sum m |v|^2
 *   out[2]     potential energy 1/2 sum m phi, phi from the last force
 *              evaluation at the current positions (self pair excluded; the
 *              tree's potential, Sec. VI.A Eq. (1)); NaN if no force has
 *              been computed for the current state
 *   out[3..5]  momentum sum m v
 *   out[6..8]  angular momentum sum m x cross v about the origin
 * Positions are the FP64 master copy when the context keeps one.  The sums
 * are folded in a fixed order (run to run identical).  Synchronises s. */
int bh_diagnostics(bh_ctx *ctx, double *out, hipStream_t s);

/* Wait for s and return the latched device status (BH_OK if clean). */
int bh_sync(bh_ctx *ctx, hipStream_t s);

typedef struct bh_stats {
    int64_t n;            /* particles of the current state */
    int64_t ncells;       /* cells of the last built tree */
    int64_t nleaves;      /* leaf cells */
    int64_t ngroups;      /* target groups */
    int64_t depth;        /* deepest level holding a cell */
    int64_t n_pp;         /* particle-particle interactions of the last walk
                             (sum over groups of npp * group size) */
    int64_t n_pc;         /* particle-cell interactions of the last walk */
    double ms_sort;       /* bounding box + keys + sort + gather of the last build */
    double ms_build;      /* octree + groups of the last build */
    double ms_moments;    /* moment pass of the last build */
    double ms_walk;       /* walk kernel of the last force evaluation */
    double ms_step;       /* whole last leapfrog_step (0 if none) */
    double ms_walk_vjp;   /* adjoint walk kernel of the last tree_force_vjp (0 if none) */
} bh_stats;

/* Fill *out (host).  Synchronises s and reports latched device status. */
int bh_stats_get(bh_ctx *ctx, bh_stats *out, hipStream_t s);

/* Arrays that bh_export can copy out, with element type and count. */
typedef enum bh_array {
    BH_ARR_KEYS = 1,        /* u64 [n]      sorted keys (Morton; Peano-Hilbert with curve = 1) */
    BH_ARR_PERM = 2,        /* u32 [n]      sorted slot -> caller index */
    BH_ARR_BOX = 3,         /* f32 [5]      lo x, y, z, side, scale */
    BH_ARR_LEVEL_START = 4, /* u32 [23]     first cell of each level; [22] = ncells */
    BH_ARR_CELL_LEVEL = 5,  /* u32 [ncells] */
    BH_ARR_CELL_PREFIX = 6, /* u64 [ncells] key >> 3 (21 - level) of the cell */
    BH_ARR_CELL_BEGIN = 7,  /* u32 [ncells] first sorted particle */
    BH_ARR_CELL_COUNT = 8,  /* u32 [ncells] */
    BH_ARR_CELL_CHILD0 = 9, /* u32 [ncells] first child (undefined for leaves) */
    BH_ARR_CELL_NCHILD = 10,/* u32 [ncells] 0 for leaves */
    BH_ARR_CELL_PARENT = 11,/* u32 [ncells] 0xffffffff for the root */
    BH_ARR_MOM_M = 12,      /* f64 [ncells] mass */
    BH_ARR_MOM_COM = 13,    /* f64 [ncells][3] centre of mass */
    BH_ARR_MOM_Q = 14,      /* f64 [ncells][6] quadrupole xx, yy, zz, xy, xz, yz */
    BH_ARR_CELL_COMF = 15,  /* f32 [ncells][4] centre of mass (FP32), r_open^2 of
                               the last force evaluation */
    BH_ARR_CELL_SIZE = 16,  /* f32 [ncells][2] cell size l, |com - centre| */
    BH_ARR_GROUP_BEGIN = 17,/* u32 [ngroups] */
    BH_ARR_GROUP_COUNT = 18,/* u32 [ngroups] */
    BH_ARR_GROUP_BOX = 19,  /* f32 [ngroups][8] centre xyz, 0, half size xyz, 0
                               (written by the walk) */
    BH_ARR_GROUP_NPP = 20,  /* u32 [ngroups] particle-particle sources of the last walk */
    BH_ARR_GROUP_NPC = 21,  /* u32 [ngroups] particle-cell sources of the last walk */
    BH_ARR_ACC_SORTED = 22, /* f32 [n][4] ax, ay, az, potential in sorted order */
    BH_ARR_BOUNDARY_FLAG = 23,  /* u32 [ncells] bit 0: in the boundary tree,
                                   bit 1: terminal (after bh_boundary) */
    BH_ARR_BOUNDARY_CELLS = 24, /* u32 [nterm] terminal boundary cells, cell order */
    BH_ARR_BOUNDARY_BOX = 25,   /* f32 [nterm][8] centre xyz, 0, widened half size
                                   xyz, 0 of each terminal cell */
    BH_ARR_LET_ORIGIN = 26,     /* u32 [let cells][2] (source index, source cell);
                                   0xffffffff for virtual cells (after bh_let_build) */
    BH_ARR_LET_NODE = 27,       /* u32 [let cells][2] internal: (first child, count);
                                   leaf: (first particle, count | 0x80000000) */
    BH_ARR_LET_COMF = 28        /* f32 [let cells][4] centre of mass, r_open^2 */
} bh_array;

/* Copy one array of the last build / walk to host memory `dst` (capacity
 * `cap_bytes`); *nbytes (may be NULL) receives the byte count.  Synchronises
 * s.  Errors: BH_EINVAL (unknown id), BH_ECAPACITY (dst too small),
 * BH_ESTATE (nothing built). */
int bh_export(bh_ctx *ctx, int array, void *dst, int64_t cap_bytes, int64_t *nbytes,
              hipStream_t s);

/* The sorted keys of the last build (Sec. III.B.1) and its permutation
 * (sorted slot -> caller index), copied to host memory: keys [n] u64 and
 * perm [n] u32, n = the built particle count (bh_stats_get); either may be
 * NULL.  Synchronises s.  Errors: BH_EINVAL (null ctx), BH_ESTATE (nothing
 * built). */
int bh_export_keys(bh_ctx *ctx, uint64_t *keys, uint32_t *perm, hipStream_t s);

/* Device views of the last built tree (Sec. I.A cells, Eq. (1) moments, the
 * walk's target groups), for callers that read the tree in place.  Every
 * pointer is device memory owned by the context, valid until the next build
 * or bh_destroy; nothing is copied. */
typedef struct bh_tree_view {
    int64_t n;                  /* particles */
    int64_t ncells;             /* cells, breadth first (level, then key) */
    int64_t ngroups;            /* target groups (or paired target sets) */
    const uint32_t *level_start;/* [23] first cell of every level 0..21, then ncells */
    const uint64_t *prefix;     /* [ncells] key >> 3 (21 - level) */
    const uint32_t *level, *begin, *count, *child0, *nchild, *parent; /* [ncells] */
    const double *M;            /* [ncells] FP64 mass */
    const double *S;            /* [ncells][3] FP64 first moment (centre of mass = S / M) */
    const double *Q;            /* [ncells][6] FP64 second moment about the centre of mass:
                                   xx, yy, zz, xy, xz, yz */
    const uint32_t *group_begin;/* [ngroups + 1] first sorted particle of every group, then n */
} bh_tree_view;

/* Fill *out with the views above (host struct).  Synchronises s to read the
 * counts.  Errors: BH_EINVAL (null ctx or out), BH_ESTATE (nothing built). */
int bh_export_tree(bh_ctx *ctx, bh_tree_view *out, hipStream_t s);

/* ---- Several spatial domains on one device (Sec. III.B) -------------------
 *
 * The paper splits the particles into one domain per GPU along the
 * space-filling curve (Sec. III.B.1), keys every domain in one global box so
 * each local tree is a branch of one global octree, and gives each domain
 * the remote cells and particles its targets need as local essential trees
 * (LETs, Sec. III.B.2).  These calls run those steps with every domain a
 * context on the same device: the forces a domain receives are its own tree
 * walk plus the walk of the remote trees, and they agree with one walk of a
 * single tree over all particles within the opening-angle error. */

/* Key every later build of ctx in the cube [lo, lo + side)^3 (host lo[3])
 * instead of the particles' own bounding box (Sec. III.B.1: the global
 * bounding box all domains share).  lo == NULL restores the own box.  A
 * particle outside the cube (x < lo or fl32(x - lo) > side on some axis)
 * latches a device status reported as BH_EINVAL by the next synchronising
 * call.  Errors: BH_EINVAL (lo not finite,
 * side <= 0 or not finite). */
int bh_set_box(bh_ctx *ctx, const float *lo, float side);

/* Cut the sorted particles of ctx into p domains along the curve
 * (Sec. III.B.1: cuts that balance the tree-walk operations, no domain more
 * than a cap above the average particle count).  Needs a force walk of the
 * current tree.  Cost of a particle: 23 npp + 65 npc of its group's last
 * walk (the operation counts of Sec. VI.A).  Cut j (host int64 cuts[p + 1],
 * cuts[0] = 0, cuts[p] = n) is the first sorted slot i at which the running
 * cost of slots [0, i) reaches j/p of the total, clamped so that no domain
 * holds more than C = floor(cap n / p) particles: cuts[j] in
 * [max(cuts[j-1], n - (p - j) C), min(cuts[j-1] + C, n)].  Domains may be
 * empty.  Computed on the device (costs, cuts and clamp), then copied to
 * cuts; synchronises s.  Errors: BH_EINVAL (p outside [1, n], cap < 1 or
 * C p < n), BH_ENOMEM (device scratch of 8 (n + p + 2) bytes), BH_ESTATE (no
 * walk since the last build). */
int bh_decompose(bh_ctx *ctx, int32_t p, float cap, int64_t *cuts, hipStream_t s);

/* The same cut by the paper's two-level sampling (Sec. III.B.1), run on the
 * host as one process would run it for p = px py processes.  Process q
 * holds the particles whose caller index i has floor(i p / n) = q.  Level
 * 1: every process draws m1 cost-weighted samples of its keys (sample j is
 * the key of its first particle, in key order, at which the running cost S
 * has 2 m1 S >= (2 j + 1) W_q, W_q its total cost; each sample weighs W_q);
 * the samples, sorted by key (ties in process order), are cut into px
 * pieces of equal weight (boundary t: the key of the first sample with the
 * weight before it >= t/px of the total).  Level 2: every process draws m2
 * samples the same way, each goes to the piece its key falls in, and each
 * piece is cut into py pieces of equal weight.  The p - 1 boundary keys
 * (host bounds [p - 1], may be NULL; a boundary with no sample past it is
 * the next level-1 boundary, else 2^64 - 1) give cut j = the first sorted
 * slot whose key is >= boundary j, clamped by the cap as in bh_decompose;
 * equal keys never straddle a cut except by the clamp.  Synchronises s.
 * Errors: as bh_decompose, and BH_EINVAL for px, py, m1 or m2 < 1 or
 * px py > min(n, 65536). */
int bh_decompose_sampled(bh_ctx *ctx, int32_t px, int32_t py, int32_t m1, int32_t m2, float cap,
                         int64_t *cuts, uint64_t *bounds, hipStream_t s);

/* Copy the particles in sorted slots [lo, hi) to device arrays in sorted
 * order: pos [hi - lo][3], vel [hi - lo][3], mass [hi - lo] and ids
 * [hi - lo] (the caller index of each); any output may be NULL.  This is
 * the particle exchange of Sec. III.B.1 for one domain.  Errors: BH_EINVAL
 * (not 0 <= lo <= hi <= n), BH_ESTATE (nothing built). */
int bh_domain_extract(bh_ctx *ctx, int64_t lo, int64_t hi, float *pos, float *vel,
                      float *mass, uint32_t *ids, hipStream_t s);

/* Forces on ctx's particles from every cell and particle of another
 * context's tree (the remote tree walked in full, Sec. III.B.2), added to
 * the caller-order device outputs acc [n][3] and pot [n] (either may be
 * NULL).  Prepares src's opening radii for theta; overwrites ctx's sorted
 * accelerations, so a later leapfrog_step recomputes the own forces.
 * Errors: BH_EINVAL (src == ctx, theta, eps, different devices), BH_ESTATE
 * (either tree not built). */
int tree_force_add(bh_ctx *ctx, bh_ctx *src, float theta, float eps, float *acc, float *pot,
                   hipStream_t s);

/* Boundary tree of ctx's tree (Sec. III.B.2, the cells on the edge of the
 * local particle set and their parents): from the root through cells of
 * more than ncrit particles, stopping at cells of at most ncrit particles,
 * at leaves, and at the deepest level L at which the boundary tree has at
 * most max_cells cells.  Its terminal cells cover every particle once; each
 * gets the tight FP32 box of its particles, centre (min + max) / 2, half
 * size (max - min) / 2 + m with m = fl32(fl32(max|lo| + side) 2^-16) from
 * the key box.  Host outputs *level and *nterm may be NULL.  Valid until the
 * next build.  Synchronises s.  Errors: BH_EINVAL (max_cells < 1),
 * BH_ESTATE (nothing built), BH_ENOMEM. */
int bh_boundary(bh_ctx *ctx, int32_t max_cells, int32_t *level, int64_t *nterm,
                hipStream_t s);

/* Local essential trees of the nsrc (0..64) remote contexts srcs (host
 * array) for ctx's targets, merged into one tree below virtual cells
 * (Sec. III.B.2); nsrc = 0 (srcs may be NULL) gives an empty one.  ctx and every source need a boundary tree and the same
 * bh_set_box.  For each source the terminal boxes of ctx's boundary tree
 * walk the source tree with the force walk's opening test for theta: if no
 * box opens a terminal cell of the source's boundary tree, that boundary
 * tree is the LET; otherwise the LET is the cells the boxes reach, opened
 * cells with all their children and opened leaves with their particles.
 * Walking the LET gives ctx's groups bit for bit the interaction lists of
 * the full source tree.  Host info [nsrc][3] (may be NULL) receives per
 * source: 1 if the boundary tree sufficed, LET cells, LET particles.  Valid
 * until ctx's next build; the LET copies the sources, which may change
 * afterwards.  Writes the sources' opening radii for theta (as their own
 * tree_force would), so no source may be in use on another stream meanwhile.
 * Synchronises s.  Errors: BH_EINVAL (nsrc, theta, a source
 * that is ctx or repeated, different boxes or devices), BH_ESTATE (missing
 * boundary tree), BH_ECAPACITY (more than 2^29 cells), BH_ENOMEM. */
int bh_let_build(bh_ctx *ctx, bh_ctx *const *srcs, int32_t nsrc, float theta, int64_t *info,
                 hipStream_t s);

/* Forces on ctx's particles from its own tree and from the merged LET (one
 * walk each, the second adding to the first), written to device outputs
 * acc [.][3] and pot [.] (either may be NULL) at row rows[i] for caller
 * index i (device u32 [n], distinct rows; NULL: row i).  theta must be the
 * LET's.  Errors: BH_EINVAL (theta, eps), BH_ESTATE (no build or no LET). */
int tree_force_let(bh_ctx *ctx, float theta, float eps, const uint32_t *rows, float *acc,
                   float *pot, hipStream_t s);

/* Static description of a status code. */
const char *bh_strerror(int status);

/* Description of the last failure on this context ("" if none). */
const char *bh_last_error(const bh_ctx *ctx);

/* Largest n of tree_force_static. */
#define BH_STATIC_MAX_N 65536

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): tree_build
 * followed by tree_force, with nleaf = 16, ncrit = 64, FP32 terms and Morton
 * keys, without a context.  Every intermediate buffer (sorted state, keys,
 * cells, moments, groups, walk stacks) lives in one static device array of
 * 64 MiB that each device the library runs on holds until the process ends;
 * the call allocates nothing (no hipMalloc, no host or device allocation by a
 * library routine).
 *   pos, mass    device, [n][3] and [n] FP32, caller order (read)
 *   n            1 .. BH_STATIC_MAX_N
 *   theta, eps   as tree_force
 *   acc, pot     device, [n][3] and [n] FP32, caller order (written; either
 *                may be NULL)
 *   status       device, one uint32_t (may be NULL): receives the device
 *                status bits of this call (1 non-finite position, 2 mass <= 0
 *                or not finite; 0 when clean), valid once s has passed it
 * Results equal those of tree_build + tree_force on a context with the same
 * parameters.  Every call on one device shares that device's array and keeps
 * the last call's contents: calls that overlap on one device (two streams,
 * two host threads) race and give undefined results; serialise them.
 * Errors: BH_EINVAL (null pos or mass, n <= 0, theta / eps out of range),
 * BH_ECAPACITY (n > BH_STATIC_MAX_N), BH_EHIP (a HIP runtime call failed).
 * There is no context, so bh_last_error has no message for this call. */
int tree_force_static(const float *pos, const float *mass, int64_t n, float theta, float eps,
                      float *acc, float *pot, uint32_t *status, hipStream_t s);

#ifdef __cplusplus
}
#endif

#endif /* BH_H */
