// Shared device-side definitions of the powersort HIP library (gfx950).
//
// Keys of every supported type are compared as unsigned "order keys": a
// bijective bit map under which unsigned integer order is the key order
// (two's-complement integers: flip the sign bit; binary32: IEEE totalOrder).
// Kernels map keys on load and map them back on store, so buffers always hold
// the caller's bit patterns.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ps {

enum KeyType : int { KT_I32 = 0, KT_U32 = 1, KT_I64 = 2, KT_U64 = 3, KT_F32 = 4 };

template <int KT> struct Key;
template <> struct Key<KT_I32> {
    using raw = uint32_t;
    using ukey = uint32_t;
    static __device__ __forceinline__ ukey ord(raw x) { return x ^ 0x80000000u; }
    static __device__ __forceinline__ raw unord(ukey u) { return u ^ 0x80000000u; }
};
template <> struct Key<KT_U32> {
    using raw = uint32_t;
    using ukey = uint32_t;
    static __device__ __forceinline__ ukey ord(raw x) { return x; }
    static __device__ __forceinline__ raw unord(ukey u) { return u; }
};
template <> struct Key<KT_I64> {
    using raw = uint64_t;
    using ukey = uint64_t;
    static __device__ __forceinline__ ukey ord(raw x) { return x ^ 0x8000000000000000ull; }
    static __device__ __forceinline__ raw unord(ukey u) { return u ^ 0x8000000000000000ull; }
};
template <> struct Key<KT_U64> {
    using raw = uint64_t;
    using ukey = uint64_t;
    static __device__ __forceinline__ ukey ord(raw x) { return x; }
    static __device__ __forceinline__ raw unord(ukey u) { return u; }
};
// binary32 totalOrder: negative values have all bits flipped, non-negative
// values get the sign bit set.
template <> struct Key<KT_F32> {
    using raw = uint32_t;
    using ukey = uint32_t;
    static __device__ __forceinline__ ukey ord(raw x) {
        return (x & 0x80000000u) ? ~x : (x | 0x80000000u);
    }
    static __device__ __forceinline__ raw unord(ukey u) {
        return (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
    }
};

// ------------------------------------------------------------- tile shapes

constexpr int kThreads = 256;       // threads per workgroup (4 wave64s)
constexpr int kWaves = kThreads / 64;

// Run partition: tiles of kPartTile positions, plus a halo of w+1 keys.
constexpr int kPartItems = 16;
constexpr int kPartTile = kThreads * kPartItems;  // 4096
constexpr int kMaxMinRun = 64;                    // largest supported w
constexpr int kScanGroup = 128;                   // tables composed per group (LDS: 128*(w+1)*5 B)

// Fused subtrees: every maximal subtree of at most kFuse elements is formed
// and merged entirely in LDS by one workgroup.
constexpr int kFuseThreads = 512;
constexpr int kFuseWaves = kFuseThreads / 64;
constexpr int kFuseItems = 8;
constexpr int kFuse = kFuseThreads * kFuseItems;  // 4096
// A fused subtree with at least this many leaves is sorted by the block
// radix sort instead of level-by-level merges (any key width: 8-byte keys
// need 108 KiB of LDS, one block per CU, and still win on permutations);
// smaller ones hold at most kFuseRadixMinLeaves - 2 merges.
constexpr uint32_t kFuseRadixMinLeaves = 8;
__host__ __device__ constexpr bool fuse_by_radix(uint32_t key_bytes, uint32_t nleaves) {
    return (key_bytes == 4 || key_bytes == 8) && nleaves >= kFuseRadixMinLeaves;
}
// The kernel that forms a fused subtree of nleaves leaves and n elements: a
// single natural run is copied (reversed if decreasing), a subtree of few
// leaves is merged level by level, one of many leaves is radix-sorted.  The
// subtrees of each kind form a list of their own.
enum UnitKind : uint32_t { kUnitCopy = 0, kUnitFew = 1, kUnitRadix = 2 };
__host__ __device__ constexpr uint32_t unit_kind(uint32_t key_bytes, uint32_t nleaves, uint32_t n) {
    return (nleaves == 1 && n > (uint32_t)kMaxMinRun) ? kUnitCopy
           : fuse_by_radix(key_bytes, nleaves)           ? kUnitRadix
                                                         : kUnitFew;
}

// Global merge passes: merge-path tiles of 8192 outputs (1024 threads x 8)
// by default for 4-byte keys, which halves the split searches; 8-byte keys
// use 4096 (1024 x 4) in place of 8192.  2048 and 4096 can be tuned for
// either.
constexpr uint32_t kMergeTileDefault = 8192;
constexpr uint32_t kMergeTileMin = 2048;
// Merges with absorbed children: splitters every kQuadSpacing positions of
// each child's merge, so a tile holds at most 2 kQuadSpacing outputs, and
// the merge pass packs consecutive tiles into groups of up to kQuadTile.
constexpr uint32_t kQuadSpacing = 2048;
constexpr uint32_t kQuadTile = 4096;
constexpr int kLog2QuadTile = 13;  // halving steps of a co-rank search over up to kQuadTile elements
// Splitter search (4-byte keys): every position divisible by kSampleSpacing
// keeps a copy of its current order key in a small sample array, so that a
// merge-path co-rank is first found among the samples (a few cached lines)
// and then within fewer than 2 kSampleSpacing positions of the runs.  The
// search is k-ary: kSplitGroup lanes probe evenly spaced points per round.
constexpr uint32_t kSampleSpacing = 128;
constexpr int kSplitGroup = 16;

// Copy/reverse of leaves longer than kFuse.
constexpr int kLeafTile = 16384;

// Where a sorted tree vertex lives.  Array 0 is the caller's, 1 and 2 are
// scratch.  A merge must not write the array it reads, so a vertex and its
// children always sit in different arrays.
//  * Two arrays: the depth parity; a long leaf at odd depth is copied to 1.
//  * Three arrays: segment roots end in 0, inner nodes alternate 2, 1, 2, ...
//    by depth, and a leaf longer than a fused subtree stays in place in 0
//    (reversed there if decreasing) unless its parent is the root, which
//    writes 0: such a leaf is copied to 2 like the root's other children.
//    This saves the copy of every long leaf at odd depth for one more
//    array of scratch.
//  * Two-level passes (a big node at odd depth merged together with its
//    parent, never written out): the same rules by "pass level"
//    (depth + 1) / 2 in place of the depth, so that every input of a merge
//    -- a child, or a grandchild through an absorbed child, all at the same
//    pass level -- sits in an array other than the merge's own.
__host__ __device__ constexpr uint32_t pass_level(uint32_t depth, uint32_t levels) {
    return levels == 2 ? (depth + 1) >> 1 : depth;
}
__host__ __device__ constexpr uint32_t node_buf(uint32_t level, uint32_t nbuf) {
    return nbuf == 3 ? (level == 0 ? 0u : 1u + (level & 1u)) : (level & 1u);
}
__host__ __device__ constexpr uint32_t big_leaf_buf(uint32_t level, uint32_t nbuf) {
    return nbuf == 3 ? (level == 1 ? 2u : 0u) : (level & 1u);
}
// The array a long leaf is copied into when it moves.
__host__ __device__ constexpr uint32_t leaf_copy_buf(uint32_t nbuf) { return nbuf == 3 ? 2u : 1u; }

constexpr int kMaxPower = 32;  // powers are at most floor(lg n) + 1 <= 32 for n < 2^31
// Merge-pass keys: node powers, or peeksort depth + 1.  A peeksort node at
// depth d >= 2 covers at most half the elements of its ancestor at depth
// d - 2, so internal nodes sit at depth <= 2 floor(lg n) - 1 and their keys
// are <= 2 floor(lg n) <= 62 for n < 2^31: the per-pass counters hold
// kMaxPass + 1 entries, and a fused subtree's 64-bit level mask covers them.
constexpr int kMaxPass = 64;

// Per-call limits.
constexpr uint64_t kMaxSegment = (1ull << 31) - 1;
// Positions are u32 in every kernel: below 2^31, a position plus any
// grid stride or tile length stays below 2^32, so no index can wrap.  A
// segmented batch above this runs as consecutive chunks of at most
// kMaxTotal elements, cut at segment boundaries.
constexpr uint64_t kMaxTotal = (1ull << 31) - 1;
constexpr uint64_t kMaxBatch = (1ull << 63) - 1;  // n_total of a segmented batch
constexpr uint64_t kMaxTreeLeaves = 1ull << 28;  // leaves of ps_alphabetic_tree

__device__ __forceinline__ int clz32(uint32_t x) { return __clz(x); }

}  // namespace ps
