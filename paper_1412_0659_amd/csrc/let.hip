// Boundary trees and local essential trees (LETs) of spatial domains
// (Sec. III.B.2: each domain cuts its tree down to the cells on the edge of
// its particle set; a remote domain checks whether that boundary tree holds
// enough cells for its own targets, and otherwise receives the specific set
// of cells and particles its targets reach; the received trees become
// branches of one tree that the force walk reads).
//
// Boundary tree of a domain: from the root through cells of more than ncrit
// particles, stopping at cells of at most ncrit particles, at leaves and at
// a level L (the deepest at which the tree has at most max_cells cells).
// Its terminal cells cover every particle once; their tight particle boxes,
// widened by a margin, stand for the domain's targets.
//
// LET of a source tree for a target domain: every target box walks the
// source tree with the force walk's own traversal and opening test.  Cells
// the boxes accept and the leaves they open are marked; a pass up the
// levels then gives, per cell, whether some box opened it and whether some
// box reached it, and marks the particles of opened leaves.  Any target group lies inside one terminal
// box, and the margin keeps its FP32 box distance to any cell at least the
// box's, so a group opens only cells that its box opens: the reached cells
// (opened cells with all their children, opened leaves with their particles)
// are exactly what the group walks need, and walking them gives bit for bit
// the interaction lists of the full source tree.  When no box opens a
// terminal cell of the source's boundary tree, the boundary tree itself
// serves as the LET.
#include "walk_common.h"

namespace bh {

uint32_t cell_count(const bh_ctx *c, hipStream_t st) {
    uint32_t nc = 0;
    if (hipStreamSynchronize(st) != hipSuccess ||
        hipMemcpy(&nc, c->cells.ls + kLevels, sizeof(uint32_t), hipMemcpyDeviceToHost) !=
            hipSuccess)
        return 0;
    return nc;
}

// ---- boundary tree ----------------------------------------------------------

__global__ __launch_bounds__(256) void k_bnd_flags(Cells c, uint32_t ncrit, uint32_t *flag,
                                                   uint32_t *lvl) {
    const uint32_t nc = c.ls[kLevels];
    const uint32_t lane = threadIdx.x & 63u;
    // every thread of a wave runs the same trips, so the counts can be
    // combined across the wave (cells are level-ordered: most waves see one level)
    for (uint32_t base = blockIdx.x * 256 + (threadIdx.x & ~63u); base < nc;
         base += gridDim.x * 256) {
        const uint32_t i = base + lane;
        bool inb = false;
        uint32_t lev = kLevels;
        if (i < nc) {
            inb = i == 0u || c.count[c.parent[i]] > ncrit;
            flag[i] = inb ? 1u : 0u;
            lev = c.level[i];
        }
        const uint32_t lev0 = shfl(lev, 0);
        if (ballot(lev != lev0 && i < nc) == 0ull) {
            const uint32_t k = (uint32_t)__popcll(ballot(inb));
            if (lane == 0 && k) atomicAdd(&lvl[lev0], k);
        } else if (inb) {
            atomicAdd(&lvl[lev], 1u);
        }
    }
}

// FP32 bounding box of every cell's particles, from the deepest level up:
// a leaf over its particles, an internal cell over its children (min and
// max are exact, so this equals the box over the particles)
__global__ __launch_bounds__(256) void k_cbox_leaf(Cells c, const float4 *__restrict__ xyzm,
                                                   float4 *__restrict__ cmin,
                                                   float4 *__restrict__ cmax) {
    const uint32_t nc = c.ls[kLevels];
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < nc; i += gridDim.x * 256) {
        if (c.nchild[i] != 0u) continue;
        const uint32_t b = c.begin[i], e = b + c.count[i];
        float4 mn = make_float4(INFINITY, INFINITY, INFINITY, 0.f);
        float4 mx = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.f);
        for (uint32_t j = b; j < e; ++j) {
            const float4 p = xyzm[j];
            mn.x = fminf(mn.x, p.x); mn.y = fminf(mn.y, p.y); mn.z = fminf(mn.z, p.z);
            mx.x = fmaxf(mx.x, p.x); mx.y = fmaxf(mx.y, p.y); mx.z = fmaxf(mx.z, p.z);
        }
        cmin[i] = mn;
        cmax[i] = mx;
    }
}

__global__ __launch_bounds__(256) void k_cbox_up(Cells c, int l, float4 *cmin, float4 *cmax) {
    const uint32_t first = c.ls[l], last = c.ls[l + 1];
    for (uint32_t i = first + blockIdx.x * 256 + threadIdx.x; i < last; i += gridDim.x * 256) {
        const uint32_t nch = c.nchild[i];
        if (nch == 0u) continue;
        const uint32_t k0 = c.child0[i];
        float4 mn = cmin[k0], mx = cmax[k0];
        for (uint32_t k = k0 + 1; k < k0 + nch; ++k) {
            const float4 a = cmin[k], b = cmax[k];
            mn.x = fminf(mn.x, a.x); mn.y = fminf(mn.y, a.y); mn.z = fminf(mn.z, a.z);
            mx.x = fmaxf(mx.x, b.x); mx.y = fmaxf(mx.y, b.y); mx.z = fmaxf(mx.z, b.z);
        }
        cmin[i] = mn;
        cmax[i] = mx;
    }
}

__global__ __launch_bounds__(256) void k_bnd_terminal(Cells c, uint32_t level, uint32_t ncrit,
                                                      uint32_t *flag, uint32_t *tscan) {
    const uint32_t nc = c.ls[kLevels];
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i <= nc; i += gridDim.x * 256) {
        if (i == nc) {
            flag[nc] = 0u;
            tscan[nc] = 0u;
            continue;
        }
        const uint32_t lev = c.level[i];
        const bool inb = (flag[i] & 1u) != 0u && lev <= level;
        const bool small = c.count[i] <= ncrit || c.nchild[i] == 0u;
        const bool term = inb && (lev == level || small);
        flag[i] = (inb ? 1u : 0u) | (term ? 2u : 0u);
        tscan[i] = term ? 1u : 0u;
    }
}

__global__ __launch_bounds__(256) void k_bnd_ids(const uint32_t *__restrict__ flag,
                                                 const uint32_t *__restrict__ tscan, uint32_t nc,
                                                 uint32_t *__restrict__ ids) {
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < nc; i += gridDim.x * 256)
        if (flag[i] & 2u) ids[tscan[i]] = i;
}

// tight FP32 box of each terminal cell: centre (min + max) / 2, half size
// (max - min) / 2 + margin
__global__ __launch_bounds__(256) void k_bnd_box(const uint32_t *__restrict__ ids, uint32_t nterm,
                                                 const float4 *__restrict__ cmin,
                                                 const float4 *__restrict__ cmax, float margin,
                                                 float4 *__restrict__ box) {
    for (uint32_t k = blockIdx.x * 256 + threadIdx.x; k < nterm; k += gridDim.x * 256) {
        const uint32_t cell = ids[k];
        const float4 mn = cmin[cell], mx = cmax[cell];
        box[2 * (size_t)k] = make_float4((mn.x + mx.x) * 0.5f, (mn.y + mx.y) * 0.5f,
                                         (mn.z + mx.z) * 0.5f, 0.f);
        box[2 * (size_t)k + 1] =
            make_float4((mx.x - mn.x) * 0.5f + margin, (mx.y - mn.y) * 0.5f + margin,
                        (mx.z - mn.z) * 0.5f + margin, 0.f);
    }
}

void launch_bnd_flags(bh_ctx *c, hipStream_t st) {
    launch_fill_u32(c->bnd.lvl, 0u, kLevels, st);
    hipLaunchKernelGGL(k_bnd_flags, dim3(kGrid), dim3(256), 0, st, c->cells,
                       (uint32_t)c->p.ncrit, c->bnd.flag, c->bnd.lvl);
}

void launch_bnd_terminal(bh_ctx *c, int level, hipStream_t st) {
    hipLaunchKernelGGL(k_bnd_terminal, dim3(kGrid), dim3(256), 0, st, c->cells, (uint32_t)level,
                       (uint32_t)c->p.ncrit, c->bnd.flag, c->bnd.scan);
}

void launch_bnd_boxes(bh_ctx *c, uint32_t nc, uint32_t nterm, hipStream_t st) {
    Boundary &b = c->bnd;
    hipLaunchKernelGGL(k_bnd_ids, dim3(kGrid), dim3(256), 0, st, (const uint32_t *)b.flag,
                       (const uint32_t *)b.scan, nc, b.ids);
    if (nterm == 0) return;
    hipLaunchKernelGGL(k_cbox_leaf, dim3(kGrid * 2), dim3(256), 0, st, c->cells,
                       (const float4 *)c->xyzm, b.cmin, b.cmax);
    for (int l = kLevels - 2; l >= 0; --l)
        hipLaunchKernelGGL(k_cbox_up, dim3(kGrid), dim3(256), 0, st, c->cells, l, b.cmin, b.cmax);
    uint32_t nb = cdiv(nterm, 256);
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_bnd_box, dim3(nb), dim3(256), 0, st, (const uint32_t *)b.ids, nterm,
                       (const float4 *)b.cmin, (const float4 *)b.cmax, b.margin, b.box);
}

// ---- local essential tree ---------------------------------------------------

// One wave per target box (grid-stride): the force walk's traversal of the
// source tree; accepted cells (cmark) and opened leaves (omark) are marked.
__global__ __launch_bounds__(64) void k_let_mark(TreeView tv, const float4 *__restrict__ tbox,
                                                 uint32_t nbox, uint32_t *cmark, uint32_t *omark,
                                                 uint32_t *spill_base) {
    __shared__ TravLds L;
    const uint32_t lane = threadIdx.x;
    uint32_t *spill = spill_base + (size_t)blockIdx.x * kStackMax;
    for (uint32_t k = blockIdx.x; k < nbox; k += gridDim.x) {
        const float4 bc = tbox[2 * (size_t)k], bh = tbox[2 * (size_t)k + 1];
        GroupBox b;
        b.cx = bc.x; b.cy = bc.y; b.cz = bc.z;
        b.hx = bh.x; b.hy = bh.y; b.hz = bh.z;
        uint32_t npc = 0, npp = 0;
        traverse<true>(
            tv, b, lane, L, spill, npc, npp,
            [&](uint32_t n) {
                for (uint32_t i = lane; i < n; i += 64u) cmark[L.pcidx[i]] = 1u;
            },
            [&](uint32_t n) {
                for (uint32_t i = lane; i < n; i += 64u) omark[L.ppidx[i]] = 1u;
            });
    }
}

// Level l, after level l + 1: opened = a marked leaf or an internal cell
// with a reached child; reached = accepted or opened.  The particles of an
// opened leaf are marked in pmark.
__global__ __launch_bounds__(256) void k_let_up(Cells c, int l, uint32_t *cmark,
                                                const uint32_t *__restrict__ omark,
                                                uint32_t *__restrict__ pmark,
                                                const uint32_t *__restrict__ bflag,
                                                uint32_t *word) {
    const uint32_t first = c.ls[l], last = c.ls[l + 1];
    for (uint32_t i = first + blockIdx.x * 256 + threadIdx.x; i < last; i += gridDim.x * 256) {
        const uint32_t acc = cmark[i] & 1u;
        const uint32_t nch = c.nchild[i];
        bool opn = false;
        if (nch == 0u) {
            opn = omark[i] != 0u;
            if (opn) {
                const uint32_t b = c.begin[i], e = b + c.count[i];
                for (uint32_t j = b; j < e; ++j) pmark[j] = 1u;
            }
        } else {
            const uint32_t k0 = c.child0[i];
            for (uint32_t k = k0; k < k0 + nch; ++k) opn = opn || (cmark[k] & 4u) != 0u;
        }
        const bool vis = acc != 0u || opn;
        cmark[i] = acc | (opn ? 2u : 0u) | (vis ? 4u : 0u);
        if (opn && (bflag[i] & 2u)) atomicOr(word, 1u);
    }
}

__global__ __launch_bounds__(256) void k_let_keep(uint32_t nc, const uint32_t *__restrict__ cmark,
                                                  const uint32_t *__restrict__ bflag,
                                                  uint32_t boundary_only, uint32_t *cscan) {
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i <= nc; i += gridDim.x * 256) {
        uint32_t keep = 0u;
        if (i < nc) keep = boundary_only ? (bflag[i] & 1u) : ((cmark[i] >> 2) & 1u);
        cscan[i] = keep;
    }
}

__global__ __launch_bounds__(256) void k_copy_flags(uint32_t n, const uint32_t *__restrict__ in,
                                                    uint32_t *out) {
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i <= n; i += gridDim.x * 256)
        out[i] = i < n ? in[i] : 0u;
}

struct LetOut {
    float4 *wA, *P0, *P1, *P2;
    uint2 *wN;
    uint32_t *origin;
    float4 *xyzm;
};

// Kept source cells -> LET slots: the root at root_slot, cell i at
// cbase + rank(i) - 1.  An expanded cell keeps its children (internal) or
// its particles (leaf); every other kept cell becomes a leaf with none.
__global__ __launch_bounds__(256) void k_let_emit(Cells c, uint32_t nc,
                                                  const uint32_t *__restrict__ cmark,
                                                  const uint32_t *__restrict__ bflag,
                                                  const uint32_t *__restrict__ cscan,
                                                  const uint32_t *__restrict__ pscan,
                                                  uint32_t boundary_only, uint32_t src_index,
                                                  uint32_t root_slot, uint32_t cbase,
                                                  uint32_t pbase, LetOut o) {
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < nc; i += gridDim.x * 256) {
        const uint32_t keep = boundary_only ? (bflag[i] & 1u) : ((cmark[i] >> 2) & 1u);
        if (!keep) continue;
        const uint32_t r = cscan[i];
        const uint32_t slot = r == 0u ? root_slot : cbase + r - 1u;
        const bool expand = boundary_only ? (bflag[i] & 3u) == 1u : (cmark[i] & 2u) != 0u;
        const uint32_t nch = c.nchild[i];
        uint2 N = make_uint2(0u, kLeafBit);
        if (expand && nch) N = make_uint2(cbase + cscan[c.child0[i]] - 1u, nch);
        else if (expand) N = make_uint2(pbase + pscan[c.begin[i]], c.count[i] | kLeafBit);
        o.wA[slot] = c.wA[i];
        o.P0[slot] = c.P0[i];
        o.P1[slot] = c.P1[i];
        o.P2[slot] = c.P2[i];
        o.wN[slot] = N;
        o.origin[2 * (size_t)slot] = src_index;
        o.origin[2 * (size_t)slot + 1] = i;
    }
}

__global__ __launch_bounds__(256) void k_let_parts(uint32_t n, const float4 *__restrict__ sxyzm,
                                                   const uint32_t *__restrict__ pmark,
                                                   const uint32_t *__restrict__ pscan,
                                                   uint32_t pbase, float4 *__restrict__ out) {
    for (uint32_t j = blockIdx.x * 256 + threadIdx.x; j < n; j += gridDim.x * 256)
        if (pmark[j]) out[pbase + pscan[j]] = sxyzm[j];
}

static uint32_t grid_for(uint64_t n) {
    uint32_t nb = cdiv(n, 256);
    if (nb > 4096) nb = 4096;
    return nb < 1 ? 1 : nb;
}

void launch_let_mark(bh_ctx *tgt, const bh_ctx *src, uint32_t nc, hipStream_t st) {
    Let &t = tgt->let;
    const uint32_t n = (uint32_t)src->n;
    launch_fill_u32(t.cmark, 0u, (uint64_t)nc + 1, st);
    launch_fill_u32(t.omark, 0u, (uint64_t)nc + 1, st);
    launch_fill_u32(t.pmark, 0u, (uint64_t)n + 1, st);
    launch_fill_u32(t.word, 0u, 1, st);
    const uint32_t nbox = tgt->bnd.nterm;
    if (nbox) {
        TreeView tv;
        tv.wA = src->cells.wA;
        tv.wN = src->cells.wN;
        tv.ring = (uint32_t)kRing;
        tv.status = tgt->status;
        const uint32_t grid = nbox < (uint32_t)tgt->walk_grid ? nbox : (uint32_t)tgt->walk_grid;
        hipLaunchKernelGGL(k_let_mark, dim3(grid), dim3(64), 0, st, tv,
                           (const float4 *)tgt->bnd.box, nbox, t.cmark, t.omark, tgt->spill);
    }
    for (int l = kLevels - 1; l >= 0; --l)
        hipLaunchKernelGGL(k_let_up, dim3(kGrid), dim3(256), 0, st, src->cells, l, t.cmark,
                           (const uint32_t *)t.omark, t.pmark, (const uint32_t *)src->bnd.flag,
                           t.word);
}

void launch_let_keep(bh_ctx *tgt, const bh_ctx *src, uint32_t nc, bool boundary_only,
                     hipStream_t st) {
    Let &t = tgt->let;
    const uint32_t n = (uint32_t)src->n;
    hipLaunchKernelGGL(k_let_keep, dim3(grid_for((uint64_t)nc + 1)), dim3(256), 0, st, nc,
                       (const uint32_t *)t.cmark, (const uint32_t *)src->bnd.flag,
                       boundary_only ? 1u : 0u, t.cscan);
    launch_exclusive_scan(t.cscan, t.cscan, nc + 1, t.spart, st);
    if (boundary_only) {
        launch_fill_u32(t.pscan, 0u, (uint64_t)n + 1, st);
    } else {
        hipLaunchKernelGGL(k_copy_flags, dim3(grid_for((uint64_t)n + 1)), dim3(256), 0, st, n,
                           (const uint32_t *)t.pmark, t.pscan);
        launch_exclusive_scan(t.pscan, t.pscan, n + 1, t.spart, st);
    }
}

void launch_let_emit(bh_ctx *tgt, const bh_ctx *src, uint32_t nc, int src_index,
                     bool boundary_only, uint32_t root_slot, uint32_t cbase, uint32_t pbase,
                     hipStream_t st) {
    Let &t = tgt->let;
    const uint32_t n = (uint32_t)src->n;
    LetOut o{t.wA, t.P0, t.P1, t.P2, t.wN, t.origin, t.xyzm};
    hipLaunchKernelGGL(k_let_emit, dim3(grid_for(nc)), dim3(256), 0, st, src->cells, nc,
                       (const uint32_t *)t.cmark, (const uint32_t *)src->bnd.flag,
                       (const uint32_t *)t.cscan, (const uint32_t *)t.pscan,
                       boundary_only ? 1u : 0u, (uint32_t)src_index, root_slot, cbase, pbase, o);
    if (!boundary_only)
        hipLaunchKernelGGL(k_let_parts, dim3(grid_for(n)), dim3(256), 0, st, n,
                           (const float4 *)src->xyzm, (const uint32_t *)t.pmark,
                           (const uint32_t *)t.pscan, pbase, t.xyzm);
}

}  // namespace bh
