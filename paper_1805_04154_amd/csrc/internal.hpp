// Internal interfaces between the translation units of the library.
#pragma once
#include "common.hpp"

namespace ps {

struct Counters {
    uint32_t r;            // number of leaves
    uint32_t nunit[3];     // fused subtrees by the kernel that forms them (UnitKind)
    uint32_t nbigleaf;     // leaves longer than kFuse
    uint32_t nbig;         // nodes longer than kFuse
    uint32_t pcount[kMaxPass + 1];  // big nodes per pass key (power, or peeksort depth + 1)
    uint32_t pfill[kMaxPass + 1];
    uint32_t pbase[kMaxPass + 1];
    uint32_t ptiles[kMaxPass + 1];  // merge tiles per pass; [0] = big-leaf tiles
    uint32_t sbase[kMaxPass + 1];   // first split record of each pass
    uint32_t peek_count[kMaxPass + 1];  // peeksort: ranges of each depth
    uint32_t pcount_q[kMaxPass + 1];    // nodes per pass with an absorbed child (last in their bucket)
    uint32_t pqfill[kMaxPass + 1];
    uint32_t ptq[kMaxPass + 1];         // first tile of those nodes within the pass
};

struct Mask2 {
    uint64_t a, b;
};

// A merge of a pass: node X = [lo, hi) with children [lo, mid) and [mid, hi).
// When a child is absorbed (two-level passes: a big child at odd depth is
// merged in the same pass as its parent, never written out), its own
// children are inputs: the left child [lo, mid) is the merge of runs
// A = [lo, m1) and B = [m1, mid), the right child of C = [mid, m2) and
// D = [m2, hi).  A child that is an input has m1 = mid (B empty) or m2 = hi
// (D empty).  The result is the stable merge of A, B, C, D in that priority
// on equal keys.
struct NodeRec {
    uint32_t lo, m1, mid, m2, hi;
    uint32_t bufs;  // arrays: result (bits 0-1), A (2-3), B (4-5), C (6-7), D (8-9)
};
__host__ __device__ constexpr bool node_is_quad(const NodeRec& R) { return R.m1 != R.mid || R.m2 != R.hi; }
// A merge tile of a pass, written by the split pass: its part of each input
// run A, B, C, D as element positions [s, e) in the run's array, where its
// output starts, and the arrays (as NodeRec.bufs).
struct SplitRec {
    uint32_t s[4];
    uint32_t e[4];
    uint32_t out;
    uint32_t bufs;
};
// Per merge tile, for packing consecutive tiles: the result positions of
// its first output (bit 31: the tile is its node's first) and one past its
// last.
struct TileSpan {
    uint32_t start;
    uint32_t end;
};
constexpr uint32_t kFirstTile = 0x80000000u;
struct UnitRec {
    uint32_t ua, ub, lo, hi;  // leaves [ua, ub) spanning elements [lo, hi)
};

struct TreeLists {
    UnitRec* unit_rec;     // three lists, one per UnitKind, from unit_base[kind]
    uint8_t* unit_par;
    uint32_t unit_base[3];
    uint32_t* bigleaf;
    uint8_t* bigleaf_mode;
    uint32_t* biglist;      // big nodes in discovery order; bit 31: the node absorbs a child
    uint32_t* bucket;       // big nodes grouped by power
    NodeRec* node_rec;      // merge record of each bucket entry
    uint32_t* bucket_tile;  // first merge tile of each bucket entry (within its pass)
    uint32_t* leaf_tile;    // first copy tile of each big leaf
    uint32_t* child_l;      // left child node of node j (when its left part has >= 2 leaves)
    uint32_t* child_r;      // right child node of node j (when its right part has >= 2 leaves)
    uint32_t nbuf;          // 2 or 3 data arrays (node_buf / big_leaf_buf)
    uint32_t levels;        // tree levels merged per pass: 1, or 2 (big nodes at odd depth absorbed)
};

struct TreeArgs {
    const void* keys;
    const uint64_t* offsets;
    uint32_t nseg;
    uint32_t rmax;
    uint32_t* starts;
    Counters* cnt;
    uint64_t* Q;
    uint8_t* P;
    uint8_t* leaf_depth;
    uint8_t* node_depth;
    Mask2* aggF;
    Mask2* aggB;
    uint64_t* inF;
    uint64_t* inB;
    uint64_t* mc;
    uint32_t* Lf;
    uint32_t* Rt;
    uint32_t* nsize;  // elements below node j
    TreeLists lists;
    uint32_t merge_tile;  // outputs per merge-path tile
    unsigned long long* prof;  // profiling element counters (nullable), indexed by PS_PROF_* group
};

// Partition: how a tile follows its chain and, for a tile with few run
// changes and breaks, the lists that define its successor function.  The
// tables pass writes one per tile; the emit pass reads it instead of the
// tile's keys unless the tile needs the per-position table.
constexpr uint32_t kWalkMax = 32;
struct TileRec {
    uint32_t x0;                // end of the natural run crossing the tile start
    uint8_t mode;               // kTileTable / kTileUniform / kTileWalk
    uint8_t t0;                 // type of the window's first pair
    uint8_t nchg, nbrk;         // list lengths (walk tiles)
    uint16_t chg[kWalkMax];     // pairs whose type differs from the previous pair's
    uint16_t brk[kWalkMax];     // break pairs
    uint8_t ctype[kWalkMax];    // type of pair chg[i]
};

struct PartitionArgs {
    const void* keys;
    uint32_t N;
    const uint64_t* offsets;
    uint32_t nseg;
    uint32_t* tile_seg;  // per partition tile: first offsets index >= the tile start (nseg > 1)
    TileRec* tile_rec;   // per partition tile
    uint32_t w;
    uint8_t* code[4];
    uint32_t* cnt[4];
    uint8_t* entry[4];
    uint32_t* offs[4];
    uint32_t ntab[4];
    int levels;
    uint32_t* starts;
    uint32_t* r_dev;
    uint32_t rmax;  // capacity of the leaf arrays
    uint32_t* samp; // 4-byte keys of a sort that moves data: the sample array to fill (else null)
};

struct MoveArgs {
    void* keys[3];      // data arrays: the caller's, then scratch (keys[2] only with three arrays)
    uint32_t* pay[3];
    const uint32_t* starts;
    const uint8_t* P;
    const uint32_t* Lf;
    const uint32_t* Rt;
    const uint8_t* node_depth;
    const Counters* cnt;
    const UnitRec* unit_rec;   // three lists, one per UnitKind, from unit_base[kind]
    const uint8_t* unit_par;
    uint32_t unit_base[3];
    const uint32_t* bigleaf;
    const uint8_t* bigleaf_mode;
    const uint32_t* bucket;
    const NodeRec* node_rec;
    const uint32_t* bucket_tile;
    const uint32_t* leaf_tile;
    SplitRec* split;
    TileSpan* span;            // split_cap entries, beside split
    uint32_t split_cap;        // capacity of split (records)
    uint32_t merge_tile;       // outputs per merge-path tile
    uint32_t leaf_copy;        // array that copied long leaves go to (leaf_copy_buf)
    uint32_t n;                // elements of the call
    uint32_t* samp;            // 4-byte keys: order key of every position divisible by kSampleSpacing (else null)
};

// Launch shape chosen by the caller (ps_set_tuning) or the defaults.
struct Tuning {
    uint32_t grid_big_leaf = 2048;
    uint32_t grid_fused = 2048;
    uint32_t grid_merge = 2048;
    uint32_t grid_split = 2048;
    uint32_t merge_tile = kMergeTileDefault;
    uint32_t merge_levels = 1;  // 1: one tree level per pass; 2: two-level passes (4-byte keys)
};

enum : uint8_t { kLeafNoop = 0, kLeafCopy = 1, kLeafRevCopy = 2, kLeafRevInPlace = 3 };

hipError_t launch_partition(int kt, const PartitionArgs& a, hipStream_t st);
hipError_t launch_init(Counters* cnt, uint64_t* mc, uint32_t nseg, hipStream_t st);
hipError_t launch_tree_cost(const TreeArgs& a, hipStream_t st);
struct PeekRange {
    uint32_t a, b, g, pad;  // leaves [a, b) of segment g
};
// Peeksort's tree, depths, node ranges and merge cost for depths below
// `levels`, in 1 + ceil(levels / 2) launches.
hipError_t launch_peek_tree(const TreeArgs& a, PeekRange* f0, PeekRange* f1, uint32_t cap, uint32_t levels,
                            hipStream_t st);
hipError_t launch_node_ranges(const TreeArgs& a, hipStream_t st);
hipError_t launch_tree_lists(int kt, const TreeArgs& a, hipStream_t st);
hipError_t launch_move_stage(int kt, bool hp, const MoveArgs& a, int stage, uint32_t p, uint32_t grid,
                             hipStream_t st, hipEvent_t ev0, hipEvent_t ev1);

}  // namespace ps
