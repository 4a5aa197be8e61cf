/*
 * bh_oracle.c -- plain CPU reference for the Barnes-Hut tree-code hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library links, includes or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code with the HIP path.
 *
 * Paper: Bedorf et al., "24.77 Pflops on a Gravitational Tree-Code to
 * Simulate the Milky Way Galaxy with 18600 GPUs" (SC14, arXiv:1412.0659).
 *
 * What is computed, step by step (each function cites the passage it
 * follows):
 *   O1 bounding box and key scale      -- Sec. III.B.1 (local bounding box
 *                                          mapped to space-filling-curve keys)
 *   O2 Morton keys                      -- Sec. III.B.1 (the paper uses
 *                                          Peano-Hilbert keys; Morton keys give
 *                                          the same octree cell set)
 *   O3 key sort                         -- done by the Python wrapper with
 *                                          numpy's stable argsort (Table II
 *                                          "Sorting SFC")
 *   O4 octree build                     -- Sec. I.A: recursive octant split
 *                                          until a cell holds at most the
 *                                          critical count (16)
 *   O5 groups                           -- target groups for the group-wise
 *                                          walk (the paper's walk serves
 *                                          warps of targets, Sec. III.A)
 *   O6 multipole moments                -- Sec. I.A / Sec. VI.A Eq. (1):
 *                                          mass, centre of mass, quadrupole
 *   O7 walk with opening angle theta    -- Sec. I.A (multipole acceptance
 *                                          criterion parameterised by theta)
 *   O8 particle-cell / particle-particle forces
 *                                       -- Sec. VI.A Eq. (1) and Eq. (2),
 *                                          with Plummer softening (Sec. IV)
 *   direct O(N^2) summation             -- Sec. I.A (the theta -> 0 limit)
 *   O7r walk of another domain's tree   -- Sec. III.B.2 (forces from a
 *                                          remote domain's tree)
 *   O-LET cells a remote domain needs   -- Sec. III.B.2 (local essential
 *                                          tree; boundary-tree sufficiency)
 *
 * Floating point: every force, potential and moment is FP64.  The steps
 * whose result is an integer (keys, tree topology, the opening decision that
 * decides the interaction lists) are taken in FP32 exactly as written, with
 * no contraction (build with -ffp-contract=off), because the GPU takes those
 * decisions in FP32.  Moments are accumulated bottom-up in the plain tree
 * order (a leaf from its particles in sorted order, a parent from its
 * children in child order), which is the upward pass of the method.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define KEY_BITS 21
#define KEY_MAXQ ((1u << KEY_BITS) - 1u)
#define NLEVELS 22 /* levels 0..21 */

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* O1 -- bounding box of the particles, cube side and key scale.
 * side = largest extent (FP32); side == 0 -> 1; scale = fl32(2^21 / side)
 * with the division done in FP64. */
void orc_bbox(int64_t n, const float *pos, float *lo3, float *side_out, float *scale_out) {
    float lo[3], hi[3];
    for (int a = 0; a < 3; ++a) lo[a] = hi[a] = pos[a];
    for (int64_t i = 1; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            float v = pos[3 * i + a];
            if (v < lo[a]) lo[a] = v;
            if (v > hi[a]) hi[a] = v;
        }
    float side = 0.0f;
    for (int a = 0; a < 3; ++a) {
        float e = hi[a] - lo[a];
        if (e > side) side = e;
    }
    if (side == 0.0f) side = 1.0f;
    for (int a = 0; a < 3; ++a) lo3[a] = lo[a];
    *side_out = side;
    *scale_out = (float)(2097152.0 / (double)side);
}

/* O2 -- 63-bit Morton key: 21 bits per axis, x the most significant bit of
 * each 3-bit digit.  q = min(trunc(fl32(fl32(x - lo) * scale)), 2^21 - 1). */
void orc_keys(int64_t n, const float *pos, const float *lo, float scale, uint64_t *keys) {
    for (int64_t i = 0; i < n; ++i) {
        uint32_t q[3];
        for (int a = 0; a < 3; ++a) {
            float t = pos[3 * i + a] - lo[a];
            float u = t * scale;
            uint32_t v = u > 0.0f ? (uint32_t)u : 0u;  /* below a given box: cell 0 */
            q[a] = v > KEY_MAXQ ? KEY_MAXQ : v;
        }
        uint64_t k = 0;
        for (int b = KEY_BITS - 1; b >= 0; --b) {
            k = (k << 3) | ((uint64_t)((q[0] >> b) & 1u) << 2) |
                ((uint64_t)((q[1] >> b) & 1u) << 1) | (uint64_t)((q[2] >> b) & 1u);
        }
        keys[i] = k;
    }
}

/* O4 -- octree from keys sorted ascending.  Level 0 is the root covering all
 * particles.  A cell at level l < 21 holding more than nleaf particles is
 * split into the non-empty runs of particles that share key >> 3(20 - l);
 * every other cell is a leaf.  Cells are numbered breadth first: all cells of
 * level l in key order, then level l + 1.  level_start[l] is the first cell
 * of level l (level_start[22] = number of cells).  Returns the number of
 * cells, or -1 if cap is too small. */
int64_t orc_build(int64_t n, const uint64_t *key, int nleaf, int64_t cap, int32_t *level,
                  uint64_t *prefix, int64_t *begin, int64_t *count, int64_t *child0,
                  int32_t *nchild, int64_t *parent, int64_t *level_start) {
    if (cap < 1) return -1;
    int64_t ncell = 1;
    level[0] = 0;
    prefix[0] = 0;
    begin[0] = 0;
    count[0] = n;
    parent[0] = -1;
    child0[0] = -1;
    nchild[0] = 0;
    level_start[0] = 0;
    for (int l = 0; l < NLEVELS; ++l) {
        int64_t first = level_start[l];
        int64_t last = ncell; /* cells of level l are [first, last) */
        level_start[l + 1] = last;
        if (l == NLEVELS - 1) break;
        int shift = 3 * (KEY_BITS - 1 - l);
        for (int64_t c = first; c < last; ++c) {
            if (count[c] <= nleaf) continue;
            child0[c] = ncell;
            int64_t i = begin[c], end = begin[c] + count[c];
            while (i < end) {
                uint64_t d = key[i] >> shift;
                int64_t j = i + 1;
                while (j < end && (key[j] >> shift) == d) ++j;
                if (ncell >= cap) return -1;
                level[ncell] = l + 1;
                prefix[ncell] = d;
                begin[ncell] = i;
                count[ncell] = j - i;
                parent[ncell] = c;
                child0[ncell] = -1;
                nchild[ncell] = 0;
                ++ncell;
                i = j;
            }
            nchild[c] = (int32_t)(ncell - child0[c]);
        }
    }
    level_start[NLEVELS] = ncell;
    return ncell;
}

/* O5 -- groups: a cell is a group iff (it holds at most ncrit particles or
 * is a leaf) and (it is the root or its parent holds more than ncrit).  The
 * groups partition the particles; listed in key order.  A group cell with
 * more than ncrit particles (only a level-21 leaf of coincident keys) is cut
 * into consecutive chunks of ncrit.  Returns the number of groups. */
static int cmp_pair(const void *a, const void *b) {
    const int64_t *x = (const int64_t *)a, *y = (const int64_t *)b;
    return (x[0] > y[0]) - (x[0] < y[0]);
}

int64_t orc_groups(int64_t ncell, const int64_t *begin, const int64_t *count,
                   const int32_t *nchild, const int64_t *parent, int ncrit, int64_t *gbeg,
                   int64_t *gcnt, int64_t *gcell) {
    int64_t ng = 0;
    int64_t *pairs = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)(ncell > 0 ? ncell : 1));
    for (int64_t c = 0; c < ncell; ++c) {
        int small = count[c] <= ncrit || nchild[c] == 0;
        int top = c == 0 || count[parent[c]] > ncrit;
        if (small && top) {
            pairs[2 * ng] = begin[c];
            pairs[2 * ng + 1] = c;
            ++ng;
        }
    }
    qsort(pairs, (size_t)ng, 2 * sizeof(int64_t), cmp_pair);
    int64_t out = 0;
    for (int64_t k = 0; k < ng; ++k) {
        int64_t c = pairs[2 * k + 1];
        for (int64_t s = 0; s < count[c]; s += ncrit) {
            gbeg[out] = begin[c] + s;
            gcnt[out] = count[c] - s < ncrit ? count[c] - s : ncrit;
            gcell[out] = c;
            ++out;
        }
    }
    free(pairs);
    return out;
}

/* Group box: tight FP32 box of the group's particles; centre and half size
 * as gc = (min + max) / 2, gh = (max - min) / 2 in FP32. */
void orc_group_boxes(int64_t ng, const int64_t *gbeg, const int64_t *gcnt, const float *x,
                     const float *y, const float *z, float *gc, float *gh) {
    for (int64_t g = 0; g < ng; ++g) {
        const float *p[3] = {x, y, z};
        for (int a = 0; a < 3; ++a) {
            float mn = p[a][gbeg[g]], mx = mn;
            for (int64_t i = gbeg[g] + 1; i < gbeg[g] + gcnt[g]; ++i) {
                if (p[a][i] < mn) mn = p[a][i];
                if (p[a][i] > mx) mx = p[a][i];
            }
            gc[3 * g + a] = (mn + mx) * 0.5f;
            gh[3 * g + a] = (mx - mn) * 0.5f;
        }
    }
}

/* Integer corner coordinates of a cell: the 3*level bits of the prefix,
 * de-interleaved per axis (x the high bit of each digit). */
/* Peano-Hilbert curve, following J. Skilling, "Programming the Hilbert
 * curve", AIP Conf. Proc. 707, 381 (2004): integer coordinates of b bits
 * per axis <-> the curve's "transposed" index, whose bits interleaved like a
 * Morton key (X[0] the high bit of each 3-bit digit) give the position along
 * the curve.  The top 3l bits of a b-bit index are the l-bit index of the
 * coordinates' top l bits, so every octree cell is one contiguous key range,
 * as under the Morton order. */
static void ph_from_axes(uint32_t X[3], int b) {
    if (b < 1) return;
    const uint32_t top = 1u << (b - 1);
    for (uint32_t Q = top; Q > 1; Q >>= 1) {
        const uint32_t P = Q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;                       /* invert the lower bits of X[0] */
            } else {
                uint32_t t = (X[0] ^ X[i]) & P;  /* swap the lower bits of X[0], X[i] */
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    X[1] ^= X[0];                                /* Gray encode */
    X[2] ^= X[1];
    uint32_t t = 0;
    for (uint32_t Q = top; Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= t;
}

static void ph_to_axes(uint32_t X[3], int b) {
    if (b < 1) return;
    const uint32_t end = 2u << (b - 1);
    uint32_t t = X[2] >> 1;                      /* Gray decode */
    X[2] ^= X[1];
    X[1] ^= X[0];
    X[0] ^= t;
    for (uint32_t Q = 2; Q != end; Q <<= 1) {
        const uint32_t P = Q - 1;
        for (int i = 2; i >= 0; --i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                uint32_t u = (X[0] ^ X[i]) & P;
                X[0] ^= u;
                X[i] ^= u;
            }
        }
    }
}

static uint64_t interleave3(const uint32_t X[3], int b) {
    uint64_t k = 0;
    for (int i = b - 1; i >= 0; --i)
        k = (k << 3) | ((uint64_t)((X[0] >> i) & 1u) << 2) | ((uint64_t)((X[1] >> i) & 1u) << 1) |
            (uint64_t)((X[2] >> i) & 1u);
    return k;
}

static void deinterleave3(uint64_t k, int b, uint32_t X[3]) {
    X[0] = X[1] = X[2] = 0;
    for (int i = b - 1; i >= 0; --i) {
        uint32_t d = (uint32_t)(k >> (3 * i)) & 7u;
        X[0] = (X[0] << 1) | (d >> 2);
        X[1] = (X[1] << 1) | ((d >> 1) & 1u);
        X[2] = (X[2] << 1) | (d & 1u);
    }
}

/* Peano-Hilbert index of n integer points q[n][3] with b bits per axis, and
 * the inverse (index -> coordinates). */
void orc_ph_index(int64_t n, const uint32_t *q, int b, uint64_t *keys) {
    for (int64_t i = 0; i < n; ++i) {
        uint32_t X[3] = {q[3 * i], q[3 * i + 1], q[3 * i + 2]};
        ph_from_axes(X, b);
        keys[i] = interleave3(X, b);
    }
}

void orc_ph_coords(int64_t n, const uint64_t *keys, int b, uint32_t *q) {
    for (int64_t i = 0; i < n; ++i) {
        uint32_t X[3];
        deinterleave3(keys[i], b, X);
        ph_to_axes(X, b);
        q[3 * i] = X[0];
        q[3 * i + 1] = X[1];
        q[3 * i + 2] = X[2];
    }
}

/* 63-bit Peano-Hilbert keys of FP32 positions, with the Morton key's
 * quantisation. */
void orc_keys_ph(int64_t n, const float *pos, const float *lo, float scale, uint64_t *keys) {
    for (int64_t i = 0; i < n; ++i) {
        uint32_t X[3];
        for (int a = 0; a < 3; ++a) {
            float t = pos[3 * i + a] - lo[a];
            float u = t * scale;
            uint32_t v = u > 0.0f ? (uint32_t)u : 0u;  /* below a given box: cell 0 */
            X[a] = v > KEY_MAXQ ? KEY_MAXQ : v;
        }
        ph_from_axes(X, KEY_BITS);
        keys[i] = interleave3(X, KEY_BITS);
    }
}

static void cell_coords(uint64_t prefix, int lev, uint64_t p[3]) {
    p[0] = p[1] = p[2] = 0;
    for (int b = lev - 1; b >= 0; --b) {
        uint64_t d = (prefix >> (3 * b)) & 7u;
        p[0] = (p[0] << 1) | ((d >> 2) & 1u);
        p[1] = (p[1] << 1) | ((d >> 1) & 1u);
        p[2] = (p[2] << 1) | (d & 1u);
    }
}

/* O6 -- multipole moments, FP64.  Leaf: M = sum m, S = sum m x,
 * com = S / M, Q = sum m s s^T with s = x - com (the quadrupole of Eq. (1):
 * the second moment about the centre of mass, not trace-free).  Parent:
 * M = sum M_c, S = sum S_c, com = S / M,
 * Q = sum (Q_c + M_c d d^T) with d = com_c - com (parallel axis).
 * Geometry: cell size l = side * 2^-level, centre = lo + (p + 1/2) l with p
 * the cell's octant decoded from its key prefix (Morton, or Peano-Hilbert
 * when curve = 1), and delta = |com - centre|.  Q is stored xx, yy, zz, xy, xz, yz.
 * Also writes the FP32 copies the opening test uses: comf, lf, deltaf. */
void orc_moments(int64_t ncell, const int32_t *level, const uint64_t *prefix,
                 const int64_t *begin, const int64_t *count, const int64_t *child0,
                 const int32_t *nchild, const float *x, const float *y, const float *z,
                 const float *m, const float *lo, float side, int curve, double *M, double *S,
                 double *com, double *Q, float *comf, float *lf, float *deltaf) {
    for (int64_t c = ncell - 1; c >= 0; --c) {
        double mm = 0.0, s[3] = {0.0, 0.0, 0.0}, q[6] = {0, 0, 0, 0, 0, 0};
        double cm[3];
        if (nchild[c] == 0) {
            for (int64_t j = begin[c]; j < begin[c] + count[c]; ++j) {
                double mj = m[j];
                mm = mm + mj;
                s[0] = s[0] + mj * (double)x[j];
                s[1] = s[1] + mj * (double)y[j];
                s[2] = s[2] + mj * (double)z[j];
            }
            for (int a = 0; a < 3; ++a) cm[a] = s[a] / mm;
            for (int64_t j = begin[c]; j < begin[c] + count[c]; ++j) {
                double mj = m[j];
                double d0 = (double)x[j] - cm[0], d1 = (double)y[j] - cm[1],
                       d2 = (double)z[j] - cm[2];
                q[0] = q[0] + (mj * d0) * d0;
                q[1] = q[1] + (mj * d1) * d1;
                q[2] = q[2] + (mj * d2) * d2;
                q[3] = q[3] + (mj * d0) * d1;
                q[4] = q[4] + (mj * d0) * d2;
                q[5] = q[5] + (mj * d1) * d2;
            }
        } else {
            for (int64_t k = child0[c]; k < child0[c] + nchild[c]; ++k) {
                mm = mm + M[k];
                for (int a = 0; a < 3; ++a) s[a] = s[a] + S[3 * k + a];
            }
            for (int a = 0; a < 3; ++a) cm[a] = s[a] / mm;
            for (int64_t k = child0[c]; k < child0[c] + nchild[c]; ++k) {
                double mk = M[k];
                double d0 = com[3 * k] - cm[0], d1 = com[3 * k + 1] - cm[1],
                       d2 = com[3 * k + 2] - cm[2];
                q[0] = q[0] + (Q[6 * k + 0] + (mk * d0) * d0);
                q[1] = q[1] + (Q[6 * k + 1] + (mk * d1) * d1);
                q[2] = q[2] + (Q[6 * k + 2] + (mk * d2) * d2);
                q[3] = q[3] + (Q[6 * k + 3] + (mk * d0) * d1);
                q[4] = q[4] + (Q[6 * k + 4] + (mk * d0) * d2);
                q[5] = q[5] + (Q[6 * k + 5] + (mk * d1) * d2);
            }
        }
        M[c] = mm;
        for (int a = 0; a < 3; ++a) {
            S[3 * c + a] = s[a];
            com[3 * c + a] = cm[a];
        }
        for (int k = 0; k < 6; ++k) Q[6 * c + k] = q[k];

        uint64_t p[3];
        if (curve == 1) {  /* the cell's octant from its Peano-Hilbert prefix */
            uint32_t X[3];
            deinterleave3(prefix[c], level[c], X);
            ph_to_axes(X, level[c]);
            p[0] = X[0]; p[1] = X[1]; p[2] = X[2];
        } else {
            cell_coords(prefix[c], level[c], p);
        }
        double lc = (double)side * ldexp(1.0, -level[c]);
        double e0 = cm[0] - ((double)lo[0] + ((double)p[0] + 0.5) * lc);
        double e1 = cm[1] - ((double)lo[1] + ((double)p[1] + 0.5) * lc);
        double e2 = cm[2] - ((double)lo[2] + ((double)p[2] + 0.5) * lc);
        double dl = sqrt((e0 * e0 + e1 * e1) + e2 * e2);
        for (int a = 0; a < 3; ++a) comf[3 * c + a] = (float)cm[a];
        lf[c] = (float)lc;
        deltaf[c] = (float)dl;
    }
}

/* Opening radius of each cell for a given theta, FP32:
 * r_open = l / theta + delta; stored squared. */
void orc_open_radius(int64_t ncell, const float *lf, const float *deltaf, float theta,
                     float *ropen2) {
    for (int64_t c = 0; c < ncell; ++c) {
        float r = lf[c] / theta + deltaf[c];
        ropen2[c] = r * r;
    }
}

/* The opening test, FP32: distance from the cell's centre of mass to the
 * group's box, accept the cell as a whole iff d^2 >= r_open^2. */
static int mac_accept(const float *cc, float ro2, const float *gc, const float *gh) {
    float d[3];
    for (int a = 0; a < 3; ++a) {
        float u = fabsf(cc[a] - gc[a]) - gh[a];
        d[a] = u > 0.0f ? u : 0.0f;
    }
    float d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    return d2 >= ro2;
}

/* O8 -- one source acting on one target, Eq. (1) and Eq. (2) with
 * r_ij = r_j - r_i and |r|^2 -> |r|^2 + eps^2.  q == NULL is a point mass. */
static void interact(const double *xi, const double *src, double mj, const double *q,
                     double eps2, double *acc, double *pot, int with_pot) {
    double d[3] = {src[0] - xi[0], src[1] - xi[1], src[2] - xi[2]};
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2;
    if (r2 == 0.0) return;
    double rinv = 1.0 / sqrt(r2);
    double rinv2 = rinv * rinv;
    double r3 = rinv * rinv2, r5 = r3 * rinv2, r7 = r5 * rinv2;
    double phi = -mj * rinv;
    double a[3] = {mj * d[0] * r3, mj * d[1] * r3, mj * d[2] * r3};
    if (q) {
        double qd[3] = {q[0] * d[0] + q[3] * d[1] + q[4] * d[2],
                        q[3] * d[0] + q[1] * d[1] + q[5] * d[2],
                        q[4] * d[0] + q[5] * d[1] + q[2] * d[2]};
        double tr = q[0] + q[1] + q[2];
        double dqd = d[0] * qd[0] + d[1] * qd[1] + d[2] * qd[2];
        phi += 0.5 * tr * r3 - 1.5 * dqd * r5;
        for (int k = 0; k < 3; ++k)
            a[k] += -1.5 * tr * d[k] * r5 - 3.0 * qd[k] * r5 + 7.5 * dqd * d[k] * r7;
    }
    if (with_pot) *pot += phi;
    for (int k = 0; k < 3; ++k) acc[k] += a[k];
}

/* O7 -- the group-wise walk.  For each listed group, breadth first from the
 * root: a cell passing the opening test is one particle-cell interaction for
 * every target of the group; a failing leaf gives its particles as
 * particle-particle sources; a failing internal cell is replaced by its
 * children.  Self pairs are evaluated but add no potential.  Counts per
 * group: npc = accepted cells, npp = particles of opened leaves (self
 * included).  Outputs are in sorted order; only the listed groups' targets
 * are written.  Optional diagnostics (may be NULL): ncov = particles covered
 * (accepted cells' counts + npp, must equal N) and nself = accepted cells
 * that hold a particle of the group (must be 0). */
static void walk_groups(int64_t nglist, const int64_t *glist, const int64_t *gbeg,
                        const int64_t *gcnt, const float *gc, const float *gh,
                        const float *tx, const float *ty, const float *tz, int remote,
                        int64_t ncell, const int64_t *begin, const int64_t *count,
                        const int64_t *child0, const int32_t *nchild, const double *M,
                        const double *com, const double *Q, const float *comf,
                        const float *ropen2, const float *x, const float *y, const float *z,
                        const float *m, double eps, double *acc, double *pot, int64_t *npp,
                        int64_t *npc, int64_t *ncov, int64_t *nself) {
    double eps2 = eps * eps;
#pragma omp parallel
    {
        int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
#pragma omp for schedule(dynamic, 4)
        for (int64_t k = 0; k < nglist; ++k) {
            int64_t g = glist[k];
            int64_t b = gbeg[g], nt = gcnt[g];
            int64_t head = 0, tail = 0, cpp = 0, cpc = 0, cov = 0, self = 0;
            for (int64_t i = b; i < b + nt; ++i) {
                acc[3 * i] = acc[3 * i + 1] = acc[3 * i + 2] = 0.0;
                pot[i] = 0.0;
            }
            queue[tail++] = 0;
            while (head < tail) {
                int64_t c = queue[head++];
                if (mac_accept(&comf[3 * c], ropen2[c], &gc[3 * g], &gh[3 * g])) {
                    ++cpc;
                    cov += count[c];
                    if (!remote && begin[c] < b + nt && b < begin[c] + count[c]) ++self;
                    for (int64_t i = b; i < b + nt; ++i) {
                        double xi[3] = {tx[i], ty[i], tz[i]};
                        interact(xi, &com[3 * c], M[c], &Q[6 * c], eps2, &acc[3 * i], &pot[i], 1);
                    }
                } else if (nchild[c] == 0) {
                    cpp += count[c];
                    for (int64_t i = b; i < b + nt; ++i) {
                        double xi[3] = {tx[i], ty[i], tz[i]};
                        for (int64_t j = begin[c]; j < begin[c] + count[c]; ++j) {
                            double xj[3] = {x[j], y[j], z[j]};
                            interact(xi, xj, m[j], NULL, eps2, &acc[3 * i], &pot[i],
                                     remote || j != i);
                        }
                    }
                } else {
                    for (int64_t ch = child0[c]; ch < child0[c] + nchild[c]; ++ch) queue[tail++] = ch;
                }
            }
            npp[g] = cpp;
            npc[g] = cpc;
            if (ncov) ncov[g] = cov + cpp;
            if (nself) nself[g] = self;
        }
        free(queue);
    }
}

void orc_walk(int64_t nglist, const int64_t *glist, const int64_t *gbeg, const int64_t *gcnt,
              const float *gc, const float *gh, int64_t ncell, const int64_t *begin,
              const int64_t *count, const int64_t *child0, const int32_t *nchild,
              const double *M, const double *com, const double *Q, const float *comf,
              const float *ropen2, const float *x, const float *y, const float *z,
              const float *m, double eps, double *acc, double *pot, int64_t *npp,
              int64_t *npc, int64_t *ncov, int64_t *nself) {
    walk_groups(nglist, glist, gbeg, gcnt, gc, gh, x, y, z, 0, ncell, begin, count, child0,
                nchild, M, com, Q, comf, ropen2, x, y, z, m, eps, acc, pot, npp, npc, ncov,
                nself);
}

/* O7r -- the same walk for the groups of one tree (targets tx, ty, tz in
 * that tree's sorted order, boxes gc, gh) through the cells and particles
 * of another tree: the forces one domain's particles receive from another
 * domain (Sec. III.B.2, the local essential tree computed in full).  No
 * pair is a self pair, so every particle-particle term adds potential. */
void orc_walk_remote(int64_t nglist, const int64_t *glist, const int64_t *gbeg,
                     const int64_t *gcnt, const float *gc, const float *gh, const float *tx,
                     const float *ty, const float *tz, int64_t ncell, const int64_t *begin,
                     const int64_t *count, const int64_t *child0, const int32_t *nchild,
                     const double *M, const double *com, const double *Q, const float *comf,
                     const float *ropen2, const float *x, const float *y, const float *z,
                     const float *m, double eps, double *acc, double *pot, int64_t *npp,
                     int64_t *npc, int64_t *ncov) {
    walk_groups(nglist, glist, gbeg, gcnt, gc, gh, tx, ty, tz, 1, ncell, begin, count, child0,
                nchild, M, com, Q, comf, ropen2, x, y, z, m, eps, acc, pot, npp, npc, ncov,
                NULL);
}

/* O-LET -- the cells of a source tree that a set of target boxes reaches
 * (Sec. III.B.2: the local essential tree a remote domain needs).  Each box
 * walks the tree from the root with the opening test of the force walk; a
 * cell it reaches is visited, a reached cell that fails the test is opened
 * (an internal cell's children are then reached; a leaf's particles are
 * needed).  vis and opn are the unions over the boxes.  Returns 1 when some
 * opened cell is flagged in bterm (a terminal cell of the source's boundary
 * tree), i.e. the boundary tree alone does not suffice; bterm may be NULL. */
int orc_let_mark(int64_t nbox, const float *bc, const float *bh, int64_t ncell,
                 const int64_t *child0, const int32_t *nchild, const float *comf,
                 const float *ropen2, const uint8_t *bterm, uint8_t *vis, uint8_t *opn) {
    int insufficient = 0;
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell > 0 ? ncell : 1));
    for (int64_t c = 0; c < ncell; ++c) vis[c] = opn[c] = 0;
    for (int64_t k = 0; k < nbox; ++k) {
        int64_t head = 0, tail = 0;
        queue[tail++] = 0;
        while (head < tail) {
            int64_t c = queue[head++];
            vis[c] = 1;
            if (mac_accept(&comf[3 * c], ropen2[c], &bc[3 * k], &bh[3 * k])) continue;
            opn[c] = 1;
            if (bterm && bterm[c]) insufficient = 1;
            for (int64_t ch = child0[c]; ch < child0[c] + nchild[c]; ++ch) queue[tail++] = ch;
        }
    }
    free(queue);
    return insufficient;
}

/* Direct O(N^2) sum for the listed targets: a_i = sum_{j != i} m_j r_ij /
 * (r_ij^2 + eps^2)^{3/2}, phi_i = -sum_{j != i} m_j / (r_ij^2 + eps^2)^{1/2}. */
void orc_direct(int64_t n, const double *pos, const double *m, int64_t nt, const int64_t *tgt,
                double eps, double *acc, double *pot) {
    double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; ++k) {
        int64_t i = tgt[k];
        double a[3] = {0, 0, 0}, p = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            interact(&pos[3 * i], &pos[3 * j], m[j], NULL, eps2, a, &p, 1);
        }
        acc[3 * k] = a[0];
        acc[3 * k + 1] = a[1];
        acc[3 * k + 2] = a[2];
        pot[k] = p;
    }
}

/* Particle-cell expansion of one cell (mass, centre of mass, quadrupole) at
 * the given targets -- Eq. (1)/(2) alone, used to pin the expansion. */
void orc_expansion(int64_t nt, const double *tpos, double mc, const double *comc,
                   const double *qc, double eps, double *acc, double *pot) {
    for (int64_t k = 0; k < nt; ++k) {
        acc[3 * k] = acc[3 * k + 1] = acc[3 * k + 2] = 0.0;
        pot[k] = 0.0;
        interact(&tpos[3 * k], comc, mc, qc, eps * eps, &acc[3 * k], &pot[k], 1);
    }
}

/* ---------------------------------------------------------------------------
 * Differentiation with frozen decisions.
 *
 * The walk's decisions (which cells each group accepts, which leaves it
 * opens) and the tree topology are recorded once and held fixed; the force
 * is then a smooth function of the positions and masses through Eq. (1)-(2)
 * and through the moments of the accepted cells.  orc_walk_record stores the
 * decisions; orc_replay evaluates the force for new (x, m) with them (FP64
 * positions, so finite differences can perturb them); orc_replay_vjp is the
 * hand-written adjoint: u -> (u^T da/dx, u^T da/dm).
 * ------------------------------------------------------------------------- */

/* Record the decisions of the walk for groups [0, ng): per group g the
 * accepted cells pc[pc_off[g] .. pc_off[g+1]) and opened leaves
 * lf[lf_off[g] .. lf_off[g+1]).  With pc == NULL only the offsets are
 * filled (counts prefix-summed), so the caller can size the lists. */
void orc_walk_record(int64_t ng, const int64_t *gbeg, const int64_t *gcnt, const float *gc,
                     const float *gh, int64_t ncell, const int64_t *child0,
                     const int32_t *nchild, const float *comf, const float *ropen2,
                     int64_t *pc_off, int64_t *pc, int64_t *lf_off, int64_t *lf) {
    (void)gbeg;
    (void)gcnt;
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
    int64_t npc = 0, nlf = 0;
    pc_off[0] = 0;
    lf_off[0] = 0;
    for (int64_t g = 0; g < ng; ++g) {
        int64_t head = 0, tail = 0;
        queue[tail++] = 0;
        while (head < tail) {
            int64_t c = queue[head++];
            if (mac_accept(&comf[3 * c], ropen2[c], &gc[3 * g], &gh[3 * g])) {
                if (pc) pc[npc] = c;
                ++npc;
            } else if (nchild[c] == 0) {
                if (lf) lf[nlf] = c;
                ++nlf;
            } else {
                for (int64_t ch = child0[c]; ch < child0[c] + nchild[c]; ++ch) queue[tail++] = ch;
            }
        }
        pc_off[g + 1] = npc;
        lf_off[g + 1] = nlf;
    }
    free(queue);
}

/* Moments of every cell from FP64 positions with a fixed topology
 * (the upward pass of orc_moments, without the FP32 copies). */
static void moments64(int64_t ncell, const int64_t *begin, const int64_t *count,
                      const int64_t *child0, const int32_t *nchild, const double *x,
                      const double *m, double *M, double *com, double *Q) {
    for (int64_t c = ncell - 1; c >= 0; --c) {
        double mm = 0.0, s[3] = {0, 0, 0}, q[6] = {0, 0, 0, 0, 0, 0}, cm[3];
        if (nchild[c] == 0) {
            for (int64_t j = begin[c]; j < begin[c] + count[c]; ++j) {
                mm += m[j];
                for (int a = 0; a < 3; ++a) s[a] += m[j] * x[3 * j + a];
            }
            for (int a = 0; a < 3; ++a) cm[a] = s[a] / mm;
            for (int64_t j = begin[c]; j < begin[c] + count[c]; ++j) {
                double d[3] = {x[3 * j] - cm[0], x[3 * j + 1] - cm[1], x[3 * j + 2] - cm[2]};
                q[0] += m[j] * d[0] * d[0];
                q[1] += m[j] * d[1] * d[1];
                q[2] += m[j] * d[2] * d[2];
                q[3] += m[j] * d[0] * d[1];
                q[4] += m[j] * d[0] * d[2];
                q[5] += m[j] * d[1] * d[2];
            }
        } else {
            for (int64_t k = child0[c]; k < child0[c] + nchild[c]; ++k) {
                mm += M[k];
                for (int a = 0; a < 3; ++a) s[a] += M[k] * com[3 * k + a];
            }
            for (int a = 0; a < 3; ++a) cm[a] = s[a] / mm;
            for (int64_t k = child0[c]; k < child0[c] + nchild[c]; ++k) {
                double d[3] = {com[3 * k] - cm[0], com[3 * k + 1] - cm[1], com[3 * k + 2] - cm[2]};
                q[0] += Q[6 * k + 0] + M[k] * d[0] * d[0];
                q[1] += Q[6 * k + 1] + M[k] * d[1] * d[1];
                q[2] += Q[6 * k + 2] + M[k] * d[2] * d[2];
                q[3] += Q[6 * k + 3] + M[k] * d[0] * d[1];
                q[4] += Q[6 * k + 4] + M[k] * d[0] * d[2];
                q[5] += Q[6 * k + 5] + M[k] * d[1] * d[2];
            }
        }
        M[c] = mm;
        for (int a = 0; a < 3; ++a) com[3 * c + a] = cm[a];
        for (int k = 0; k < 6; ++k) Q[6 * c + k] = q[k];
    }
}

/* Force with frozen decisions at FP64 positions x[n][3] (sorted order) and
 * masses m[n].  M, com, Q are caller scratch of ncell entries. */
void orc_replay(int64_t ng, const int64_t *gbeg, const int64_t *gcnt, int64_t ncell,
                const int64_t *begin, const int64_t *count, const int64_t *child0,
                const int32_t *nchild, const int64_t *pc_off, const int64_t *pc,
                const int64_t *lf_off, const int64_t *lf, const double *x, const double *m,
                double eps, double *M, double *com, double *Q, double *acc, double *pot) {
    moments64(ncell, begin, count, child0, nchild, x, m, M, com, Q);
    double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t g = 0; g < ng; ++g) {
        for (int64_t i = gbeg[g]; i < gbeg[g] + gcnt[g]; ++i) {
            double a[3] = {0, 0, 0}, p = 0.0;
            for (int64_t k = pc_off[g]; k < pc_off[g + 1]; ++k) {
                int64_t c = pc[k];
                interact(&x[3 * i], &com[3 * c], M[c], &Q[6 * c], eps2, a, &p, 1);
            }
            for (int64_t k = lf_off[g]; k < lf_off[g + 1]; ++k) {
                int64_t c = lf[k];
                for (int64_t j = begin[c]; j < begin[c] + count[c]; ++j)
                    interact(&x[3 * i], &x[3 * j], m[j], NULL, eps2, a, &p, j != i);
            }
            for (int a3 = 0; a3 < 3; ++a3) acc[3 * i + a3] = a[a3];
            pot[i] = p;
        }
    }
}

/* Adjoint of one particle-cell term F(d; M, Q) of Eq. (2), d = com - x_i:
 * given the cotangent u of the acceleration, returns w = J^T u with
 * J = dF/dd, and the cotangents of M (gM) and of the six stored Q entries
 * (gQ: xx, yy, zz, xy, xz, yz).  Point masses: q == NULL. */
static void term_vjp(const double *d, double mj, const double *q, double eps2, const double *u,
                     double *w, double *gM, double *gQ) {
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2;
    if (r2 == 0.0) {
        w[0] = w[1] = w[2] = 0.0;
        *gM = 0.0;
        if (gQ)
            for (int k = 0; k < 6; ++k) gQ[k] = 0.0;
        return;
    }
    double ri = 1.0 / sqrt(r2), ri2 = ri * ri;
    double r3 = ri * ri2, r5 = r3 * ri2, r7 = r5 * ri2, r9 = r7 * ri2;
    double ud = u[0] * d[0] + u[1] * d[1] + u[2] * d[2];
    /* monopole: F = M d r^-3;  J = M (I r^-3 - 3 d d^T r^-5) */
    for (int a = 0; a < 3; ++a) w[a] = mj * (u[a] * r3 - 3.0 * d[a] * ud * r5);
    *gM = ud * r3;
    if (!q) return;
    double Qm[3][3] = {{q[0], q[3], q[4]}, {q[3], q[1], q[5]}, {q[4], q[5], q[2]}};
    double tr = q[0] + q[1] + q[2];
    double qd[3], qu[3];
    for (int a = 0; a < 3; ++a) {
        qd[a] = Qm[a][0] * d[0] + Qm[a][1] * d[1] + Qm[a][2] * d[2];
        qu[a] = Qm[a][0] * u[0] + Qm[a][1] * u[1] + Qm[a][2] * u[2];
    }
    double dqd = d[0] * qd[0] + d[1] * qd[1] + d[2] * qd[2];
    double uqd = u[0] * qd[0] + u[1] * qd[1] + u[2] * qd[2];
    /* F = -3/2 tr d r^-5 - 3 Q d r^-5 + 15/2 (d^T Q d) d r^-7
     * dF_a/dd_b:
     *   -3/2 tr (delta_ab r^-5 - 5 d_a d_b r^-7)
     *   -3 (Q_ab r^-5 - 5 (Qd)_a d_b r^-7)
     *   +15/2 (2 (Qd)_b d_a r^-7 + dqd delta_ab r^-7 - 7 dqd d_a d_b r^-9)
     * w_b = sum_a u_a dF_a/dd_b */
    for (int b = 0; b < 3; ++b) {
        double t = 0.0;
        t += -1.5 * tr * (u[b] * r5 - 5.0 * ud * d[b] * r7);
        t += -3.0 * (qu[b] * r5 - 5.0 * uqd * d[b] * r7);
        t += 7.5 * (2.0 * ud * qd[b] * r7 + dqd * u[b] * r7 - 7.0 * dqd * ud * d[b] * r9);
        w[b] += t;
    }
    /* dF/dQ_ab for the symmetric matrix, per stored entry:
     *   from -3/2 tr d r^-5: diagonal entries give -3/2 d r^-5
     *   from -3 Q d r^-5:    entry (a,b) gives -3 r^-5 (e_a d_b + e_b d_a) for a != b,
     *                        -3 r^-5 e_a d_a for a == b
     *   from 15/2 dQd d r^-7: entry gives 15/2 r^-7 d (d_a d_b (2 if a != b)) */
    static const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
    for (int k = 0; k < 6; ++k) {
        int a = ia[k], b = ib[k];
        double g = 0.0;
        if (a == b) {
            g += -1.5 * ud * r5;
            g += -3.0 * r5 * u[a] * d[a];
            g += 7.5 * r7 * ud * d[a] * d[a];
        } else {
            g += -3.0 * r5 * (u[a] * d[b] + u[b] * d[a]);
            g += 7.5 * r7 * ud * 2.0 * d[a] * d[b];
        }
        gQ[k] = g;
    }
}

/* Adjoint of orc_replay's accelerations: given u[n][3] (sorted order),
 * accumulate gx[n][3] += u^T da/dx and gm[n] += u^T da/dm.  Cell adjoints
 * (lM, lcom[3], lQ[6] per cell) are caller scratch; moments must hold the
 * replay's moments for (x, m).  Source terms are reduced serially. */
void orc_replay_vjp(int64_t ng, const int64_t *gbeg, const int64_t *gcnt, int64_t ncell,
                    const int64_t *begin, const int64_t *count, const int64_t *child0,
                    const int32_t *nchild, const int64_t *pc_off, const int64_t *pc,
                    const int64_t *lf_off, const int64_t *lf, const double *x, const double *m,
                    double eps, const double *M, const double *com, const double *Q,
                    const double *u, double *lM, double *lcom, double *lQ, double *gx,
                    double *gm) {
    (void)child0;
    (void)nchild;
    double eps2 = eps * eps;
    for (int64_t c = 0; c < ncell; ++c) {
        lM[c] = 0.0;
        for (int a = 0; a < 3; ++a) lcom[3 * c + a] = 0.0;
        for (int k = 0; k < 6; ++k) lQ[6 * c + k] = 0.0;
    }
    for (int64_t g = 0; g < ng; ++g) {
        for (int64_t i = gbeg[g]; i < gbeg[g] + gcnt[g]; ++i) {
            const double *ui = &u[3 * i];
            for (int64_t k = pc_off[g]; k < pc_off[g + 1]; ++k) {
                int64_t c = pc[k];
                double d[3] = {com[3 * c] - x[3 * i], com[3 * c + 1] - x[3 * i + 1],
                               com[3 * c + 2] - x[3 * i + 2]};
                double w[3], gM, gQ[6];
                term_vjp(d, M[c], &Q[6 * c], eps2, ui, w, &gM, gQ);
                for (int a = 0; a < 3; ++a) {
                    gx[3 * i + a] -= w[a];
                    lcom[3 * c + a] += w[a];
                }
                lM[c] += gM;
                for (int q = 0; q < 6; ++q) lQ[6 * c + q] += gQ[q];
            }
            for (int64_t k = lf_off[g]; k < lf_off[g + 1]; ++k) {
                int64_t c = lf[k];
                for (int64_t j = begin[c]; j < begin[c] + count[c]; ++j) {
                    if (j == i) continue;
                    double d[3] = {x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1],
                                   x[3 * j + 2] - x[3 * i + 2]};
                    double w[3], gM;
                    term_vjp(d, m[j], NULL, eps2, ui, w, &gM, NULL);
                    for (int a = 0; a < 3; ++a) {
                        gx[3 * i + a] -= w[a];
                        gx[3 * j + a] += w[a];
                    }
                    gm[j] += gM;
                }
            }
        }
    }
    /* moments: each particle receives the adjoints of every cell holding it
     * (its ancestors), with s = x_k - com_c:
     *   d com / d x_k = m_k / M;  d com / d m_k = s / M;  d M / d m_k = 1;
     *   d Q / d x_k = m_k (e s^T + s e^T) (the com dependence cancels since
     *   sum m s = 0);  d Q / d m_k = s s^T. */
    for (int64_t c = 0; c < ncell; ++c) {
        if (lM[c] == 0.0 && lcom[3 * c] == 0.0 && lcom[3 * c + 1] == 0.0 &&
            lcom[3 * c + 2] == 0.0) {
            int any = 0;
            for (int q = 0; q < 6; ++q) any |= lQ[6 * c + q] != 0.0;
            if (!any) continue;
        }
        const double *lq = &lQ[6 * c];
        for (int64_t k = begin[c]; k < begin[c] + count[c]; ++k) {
            double s[3] = {x[3 * k] - com[3 * c], x[3 * k + 1] - com[3 * c + 1],
                           x[3 * k + 2] - com[3 * c + 2]};
            double Ls[3] = {2.0 * lq[0] * s[0] + lq[3] * s[1] + lq[4] * s[2],
                            lq[3] * s[0] + 2.0 * lq[1] * s[1] + lq[5] * s[2],
                            lq[4] * s[0] + lq[5] * s[1] + 2.0 * lq[2] * s[2]};
            for (int a = 0; a < 3; ++a)
                gx[3 * k + a] += m[k] / M[c] * lcom[3 * c + a] + m[k] * Ls[a];
            double sLs = lq[0] * s[0] * s[0] + lq[1] * s[1] * s[1] + lq[2] * s[2] * s[2] +
                         lq[3] * s[0] * s[1] + lq[4] * s[0] * s[2] + lq[5] * s[1] * s[2];
            gm[k] += lM[c] + (lcom[3 * c] * s[0] + lcom[3 * c + 1] * s[1] +
                              lcom[3 * c + 2] * s[2]) / M[c] + sLs;
        }
    }
}
