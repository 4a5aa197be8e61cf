// Internal declarations of the gfx950 tree-code library: the context that
// owns every device buffer, and the host-side launchers each .hip file
// provides.  Every kernel is enqueued on the caller's stream; nothing here
// synchronises except where a launcher says so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "bh.h"

namespace bh {

constexpr int kKeyBits = 21;            // bits per axis of a Morton key
constexpr int kLevels = 22;             // levels 0..21
constexpr int kLsSize = 24;             // level_start entries (23 used)
constexpr int kGrid = 1024;             // fixed grid of the per-level moment, box and flag kernels
constexpr int kBuildGrid = 2048;        // grid of the octree level kernels: 8 waves per SIMD
constexpr int kTableLevel = 7;          // the build looks up the child bounds of levels < 7
constexpr uint32_t kLeafBit = 0x80000000u;
constexpr uint32_t kNone = 0xffffffffu;
constexpr int kStackMax = 2689;         // walk stack bound: 21 levels x 128 ranges + root
// Adjoint: the cells of the top levels (the first kHotCells in level order) are hit by far
// more groups than the rest, so their accumulators come in kHotCopies copies (4 per XCD).
// Field and copy strides (in doubles) are one 128-byte line more than a power-of-two
// multiple, so that the copies and fields of a cell fall on different L2 channels.
constexpr uint32_t kHotCells = 65536;
constexpr uint32_t kHotCopies = 32;
constexpr uint64_t kHotField = kHotCells + 16;
constexpr uint64_t kHotCopy = 10 * kHotField + 16;
constexpr int kDiagN = 9;               // diagnostics: M, KE, PE, p xyz, L xyz
constexpr int kDiagBlocks = 1024;       // blocks of the diagnostics reduction

// device status word bits
constexpr uint32_t kStNonFinite = 1u;
constexpr uint32_t kStMass = 2u;
constexpr uint32_t kStOverflow = 4u;
constexpr uint32_t kStIndex = 8u;       // a target index outside [0, n)
constexpr uint32_t kStOutside = 16u;    // a particle outside the caller-given key box

// Particle state in sorted (Morton) order, structure of arrays.
struct State {
    float *x, *y, *z, *m, *vx, *vy, *vz;
    uint32_t *cid;  // caller index of each sorted slot
    double *x64, *y64, *z64;  // FP64 master positions (pos_fp64 contexts), else null
};

// Octree cells, breadth-first order (level, then key).
struct Cells {
    uint64_t *prefix;  // key >> 3 (21 - level)
    uint32_t *level, *begin, *count, *child0, *nchild, *parent;
    uint32_t *ls;      // [kLsSize] level_start on the device
    uint32_t *part;    // [kBuildGrid + 1] per-block partials of the level scans
    uint32_t *lbt;     // [8^kTableLevel + 1] first sorted slot of every level-kTableLevel prefix
    uint32_t *cbnd;    // [n_max][8] child bounds 1..8 of the cells of the level being split
                       // (level-local index), from the count pass to the write pass
    // FP64 moments of the upward pass
    double *M, *S, *com, *Q;  // [c], [c][3], [c][3], [c][6]; com = S / M, filled for export
    // records read by the walk
    float4 *wA;  // com (FP32) and r_open^2 of the last theta
    uint2 *wN;   // internal: (child0, nchild); leaf: (begin, count | kLeafBit)
    float4 *P0;  // particle-cell record: com x, y, z, M
    float4 *P1;  // -3 Qxx, -3 Qyy, -3 Qzz, -3 Qxy
    float4 *P2;  // -3 Qxz, -3 Qyz, trace(Q) / 2, -3 trace(Q) / 2
    float2 *size;  // cell size l, |com - geometric centre|
};

struct Groups {
    uint32_t *flag, *scan;  // [n] group-start flags and their exclusive scan
    uint32_t *begin;        // [n + 1]
    uint32_t *count_dev;    // [1] number of groups
    float4 *box;            // [2 * n] centre, half size
    uint32_t *npp, *npc;    // [n]
};

// Boundary tree of a domain (Sec. III.B.2): the cells reached from the root
// through cells of more than ncrit particles, down to level `level`;
// terminal cells (level `level`, at most ncrit particles, or leaves) cover
// every particle once.
struct Boundary {
    bool valid = false;
    int level = -1;
    uint32_t nterm = 0;
    float margin = 0.f;        // widening of the terminal boxes
    uint32_t *flag = nullptr;  // [cap_cells + 1] bit 0: in the boundary tree, bit 1: terminal
    uint32_t *scan = nullptr;  // [cap_cells + 1] exclusive scan of the terminal bits
    uint32_t *ids = nullptr;   // [cap_cells] terminal cells in cell order
    float4 *box = nullptr;     // [2 cap_cells] centre, half size (widened) of each
    float4 *cmin = nullptr, *cmax = nullptr;  // [cap_cells] FP32 particle box of every cell
    uint32_t *lvl = nullptr;   // [kLevels] boundary cells per level
    uint32_t *part = nullptr;  // scan partials
};

// Local essential trees of remote domains merged under virtual cells
// (Sec. III.B.2), plus the scratch of their construction.
struct Let {
    bool valid = false;
    float theta = 0.f;
    int nsrc = 0;
    uint32_t ncell = 0, npart = 0;
    int64_t cell_cap = 0, part_cap = 0;
    float4 *wA = nullptr, *P0 = nullptr, *P1 = nullptr, *P2 = nullptr, *xyzm = nullptr;
    uint2 *wN = nullptr;
    uint32_t *origin = nullptr;  // [cell_cap][2] (source, source cell); kNone for virtual
    // per-source scratch, sized to the largest source
    int64_t scr_cells = 0, scr_parts = 0, part_len = 0;
    uint32_t *cmark = nullptr;  // [cells + 1] bit 0 accepted, 1 opened, 2 reached
    uint32_t *omark = nullptr;  // [cells + 1] leaves some box opened
    uint32_t *cscan = nullptr;  // [cells + 1] kept cells, scanned
    uint32_t *pmark = nullptr;  // [parts + 1] particles of opened leaves
    uint32_t *pscan = nullptr;  // [parts + 1]
    uint32_t *spart = nullptr;  // scan partials
    uint32_t *word = nullptr;   // [1] a terminal boundary cell was opened
};

// Device buffers of the domain cut: group-start costs and the cuts.
struct Cut {
    uint64_t *S = nullptr;  // [n + 1]
    int64_t *cuts = nullptr;  // [p + 1]
    int64_t S_cap = 0, cuts_cap = 0;
};

struct Sort {
    uint64_t *key[2];
    uint32_t *idx[2];
    uint32_t *counts;      // [256 * tiles]
    uint32_t *scan_part;   // partials of the generic scan
    int64_t counts_len, scan_part_len;
};

}  // namespace bh

struct bh_ctx {
    int64_t nmax = 0, cap_cells = 0, n = 0;
    bh_params p{};
    int device = 0;
    int cus = 0;

    bh::State st[2]{};
    int cur = 0;
    float4 *acc = nullptr;  // sorted acceleration + potential
    float4 *xyzm = nullptr; // sorted position + mass, one record per particle
    uint32_t *spill = nullptr;  // walk stack spill area, kStackMax per wave
    float *box = nullptr;   // [8]: lo xyz, side, scale
    float *box_part = nullptr;
    uint32_t *status = nullptr;
    uint32_t *work = nullptr;                // [8] walk work counters
    unsigned long long *totals = nullptr;    // [4] n_pp, n_pc, leaves
    bh::Sort sort{};
    bh::Cells cells{};
    bh::Groups groups{};

    // adjoint buffers (contexts created with adjoint = 1)
    // per-XCD copies (8), field-major: [8][10][cap_cells] dL/dM, dL/dcom xyz, dL/dQ xx yy zz
    // xy xz yz; [8][4][n_max] dL/dx xyz, dL/dm of sorted particles; the first kHotCells
    // cells accumulate in kHotCopies copies of kHotCopy doubles (field stride kHotField) instead
    double *lcell = nullptr;
    double *gsrc = nullptr;
    double *lhot = nullptr;
    float4 *usort = nullptr;   // [n] cotangent of the accelerations, sorted order
    uint32_t *leafof = nullptr;  // [n] leaf cell of each sorted particle
    double *cic = nullptr;       // [65536] accumulator of the surface-density grid
    uint32_t *inv = nullptr;     // [n] sorted slot of each caller index (direct sum)
    double *diag = nullptr;      // [kDiagBlocks + 1][kDiagN] diagnostics partials, result
    uint8_t *seg = nullptr;      // recomputed states of an adjoint segment (grown on demand)
    int64_t seg_cap = 0;         // bytes of seg

    bh::Boundary bnd{};
    bh::Let let{};
    bh::Cut cut{};

    // level starts of a recent build, written by k_build_tail into pinned host
    // memory: [0] build number (written first), [1] build number (written
    // last), [2 ..] ls[0 .. kLevels]
    uint32_t *hint_host = nullptr;
    uint32_t *hint_dev = nullptr;  // the same memory as the device addresses it
    uint32_t build_gen = 0;     // builds launched so far
    uint32_t hint_gen_min = 1;  // first build of the current particle set

    bool built = false, have_acc = false;
    bool counts_valid = false;  // npp / npc / totals describe a walk of the current groups
    bool fixed_box = false;     // keys relative to a caller-given box (bh_set_box)
    float box_lo[3] = {0.f, 0.f, 0.f}, box_side = 1.f;
    float acc_theta = 0.f, acc_eps = 0.f;
    int walk_grid = 0;
    bool walk_small_stack = false;  // test hook: at most 192 resident stack entries
    int forced_grid_levels = -1;    // test hook: levels split by the grid kernels
    uint32_t pair_groups = 0;       // sibling groups of together <= this many walk as one (0: off)

    // events: build start, after sort, after octree+groups, after moments,
    // walk start, walk end, step start, step end, adjoint walk start, end
    hipEvent_t ev[10]{};
    bool ev_rec[10]{};
    std::string last_error;
};

namespace bh {

// walk_vjp.hip: coef * u^T d(acc)/d(x, m) accumulated into caller-order
// g_pos [n][3] / g_mass [n] (either may be null); u is caller order [n][3]
void launch_walk_vjp(bh_ctx *c, float eps, const float *u, float coef, float *g_pos,
                     float *g_mass, hipStream_t st);
void launch_axpy3(const float *x, float *y, float a, uint32_t n, hipStream_t st);

// loss.hip: cloud-in-cell surface density on a polar grid and its adjoint
void launch_cic(const float *pos, const float *mass, const uint8_t *sel, uint32_t n, float rmin,
                float rmax, int nr, int nphi, double *scratch, float *density, hipStream_t st);
void launch_cic_vjp(const float *pos, const float *mass, const uint8_t *sel, uint32_t n,
                    float rmin, float rmax, int nr, int nphi, const float *gden, float *g_pos,
                    float *g_mass, hipStream_t st);

// direct.hip: FP64 direct sum at caller-index targets tgt [nt] (device)
// into acc [nt][3] / pot [nt] (device, FP64)
// (targets outside [0, n) are skipped and latch kStIndex)
void launch_direct(bh_ctx *c, const int64_t *tgt, uint32_t nt, float eps, double *acc,
                   double *pot, hipStream_t st);

// keys_sort.hip
void launch_bbox(bh_ctx *c, const State &s, uint32_t n, hipStream_t st);
void launch_keys(bh_ctx *c, const State &s, uint32_t n, hipStream_t st);
void launch_radix_sort(bh_ctx *c, uint32_t n, hipStream_t st);  // result in key[0], idx[0]
void launch_gather(bh_ctx *c, uint32_t n, hipStream_t st);      // st[cur] -> st[cur ^ 1]
int64_t sort_counts_len(int64_t nmax);
int64_t scan_part_len(int64_t n);

// scan.hip: exclusive scan of n u32 (in may equal out); part >= scan_part_len(n)
void launch_exclusive_scan(const uint32_t *in, uint32_t *out, uint32_t n, uint32_t *part,
                           hipStream_t st);

// build.hip
void launch_build(bh_ctx *c, uint32_t n, hipStream_t st, int grid_levels);
void launch_groups(bh_ctx *c, uint32_t n, hipStream_t st);

// moments.hip
void launch_moments(bh_ctx *c, hipStream_t st, int grid_levels);
void launch_com(bh_ctx *c, hipStream_t st);
void launch_walk_prep(bh_ctx *c, float theta, hipStream_t st);

// let.hip: boundary trees and local essential trees (Sec. III.B.2); nc is
// the cell count of the tree the launcher reads (cell_count)
void launch_bnd_flags(bh_ctx *c, hipStream_t st);                // -> bnd.flag bit 0, bnd.lvl
void launch_bnd_terminal(bh_ctx *c, int level, hipStream_t st);  // -> flag bit 1, scan input
void launch_bnd_boxes(bh_ctx *c, uint32_t nc, uint32_t nterm, hipStream_t st);  // -> ids, box
void launch_let_mark(bh_ctx *tgt, const bh_ctx *src, uint32_t nc, hipStream_t st);
void launch_let_keep(bh_ctx *tgt, const bh_ctx *src, uint32_t nc, bool boundary_only,
                     hipStream_t st);
void launch_let_emit(bh_ctx *tgt, const bh_ctx *src, uint32_t nc, int src_index,
                     bool boundary_only, uint32_t root_slot, uint32_t cbase, uint32_t pbase,
                     hipStream_t st);
uint32_t cell_count(const bh_ctx *c, hipStream_t st);  // synchronises st, reads the count

// walk.hip
// The cells and particles a walk reads: a context's own tree, another
// domain's tree, or a merged local essential tree.
struct SrcView {
    const float4 *wA;   // com, r_open^2 (prepared for the walk's theta)
    const uint2 *wN;    // internal: (child0, nchild); leaf: (first, count | kLeafBit)
    const float4 *P0, *P1, *P2;
    const float4 *xyzm;  // particles the leaves index
};
SrcView own_view(const bh_ctx *c);
void launch_walk(bh_ctx *c, float eps, hipStream_t st);
// c's groups walk the tree v; remote: no self pairs (v is not c's own tree);
// accum: forces and counts add to c->acc, npp, npc
void launch_walk_view(bh_ctx *c, const SrcView &v, float eps, bool remote, bool accum,
                      hipStream_t st);
int walk_blocks_per_cu();

// integrate.hip
void launch_ingest(bh_ctx *c, const float *pos, const float *vel, const float *mass, uint32_t n,
                   hipStream_t st);
void launch_kick(bh_ctx *c, float h, uint32_t n, hipStream_t st);
void launch_kick_drift(bh_ctx *c, float h, float dt, uint32_t n, hipStream_t st);
void launch_unsort(bh_ctx *c, float *acc, float *pot, uint32_t n, hipStream_t st,
                   const uint32_t *rows = nullptr);
void launch_unsort_add(bh_ctx *c, float *acc, float *pot, uint32_t n, hipStream_t st);
void launch_state_out(bh_ctx *c, float *pos, float *vel, uint32_t n, hipStream_t st);
void launch_range_out(bh_ctx *c, uint32_t lo, uint32_t cnt, float *pos, float *vel, float *mass,
                      uint32_t *ids, hipStream_t st);
void launch_totals(bh_ctx *c, uint32_t n, hipStream_t st);
void launch_count_leaves(bh_ctx *c, hipStream_t st);
void launch_diagnostics(bh_ctx *c, hipStream_t st);  // result at diag + kDiagBlocks * kDiagN
void launch_fill_u32(uint32_t *p, uint32_t v, uint64_t n, hipStream_t st);
void launch_cut(bh_ctx *c, int32_t p, int64_t C, uint64_t *S, int64_t *cuts, hipStream_t st);

inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// Record timing event k of the context on st (contexts without events, such
// as the one tree_force_static assembles over its static buffer, skip it).
inline void record_event(bh_ctx *c, int k, hipStream_t st) {
    if (!c->ev[k]) return;
    (void)hipEventRecord(c->ev[k], st);
    c->ev_rec[k] = true;
}

// Peano-Hilbert curve (the curve of Sec. III.B.1), after J. Skilling,
// "Programming the Hilbert curve", AIP Conf. Proc. 707, 381 (2004): integer
// coordinates of b bits per axis are turned in place into the curve's
// transposed index, whose bits interleaved like a Morton key (X[0] the high
// bit of each digit) are the position along the curve; ph_decode inverts it.
// The top 3l bits of a key are the l-bit key of the coordinates' top l bits,
// so each octree cell is one key range, as with Morton keys.
__device__ __forceinline__ void ph_encode(uint32_t X[3], int b) {
    if (b < 1) return;
    const uint32_t top = 1u << (b - 1);
    for (uint32_t Q = top; Q > 1u; Q >>= 1) {
        const uint32_t P = Q - 1u;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const uint32_t sw = (X[0] ^ X[i]) & P;
            const bool inv = (X[i] & Q) != 0u;
            X[0] ^= inv ? P : sw;      // invert the low bits of X[0], or swap them
            if (!inv) X[i] ^= sw;      //   with those of X[i]
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t t = 0;
    for (uint32_t Q = top; Q > 1u; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1u;
    X[0] ^= t;
    X[1] ^= t;
    X[2] ^= t;
}

__device__ __forceinline__ void ph_decode(uint32_t X[3], int b) {
    if (b < 1) return;
    const uint32_t end = 2u << (b - 1);
    const uint32_t t = X[2] >> 1;
    X[2] ^= X[1];
    X[1] ^= X[0];
    X[0] ^= t;
    for (uint32_t Q = 2; Q != end; Q <<= 1) {
        const uint32_t P = Q - 1u;
#pragma unroll
        for (int i = 2; i >= 0; --i) {
            const uint32_t sw = (X[0] ^ X[i]) & P;
            const bool inv = (X[i] & Q) != 0u;
            X[0] ^= inv ? P : sw;
            if (!inv) X[i] ^= sw;
        }
    }
}

}  // namespace bh
