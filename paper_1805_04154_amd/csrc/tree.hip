// Node powers and the merge tree.
//
// Leaves i = 0..r-1 (after the min-run extension) have starts S_i; boundary j
// (1 <= j < r) separates leaves j-1 and j.  Per Def. "Node Power" the power of
// boundary j is the first bit in which the binary fractions of the two run
// midpoints differ.  With q_i = floor((2 (S_i - off) + L_i) 2^32 / (2 n)), the
// 32-bit fixed-point midpoint of leaf i in its segment (origin off, length n),
// P_j = clz32(q_{j-1} xor q_j) + 1: the fixed point agrees with the exact
// definition because midpoints of adjacent leaves differ by at least 1/n > 2^-31.
// Each leaf stores Q_i = (segment << 32) | q_i, strictly increasing over the
// whole batch; a boundary between segments gets power 0.
//
// By Cor. "Cartesian tree" the merge tree is the min-oriented Cartesian tree
// of the powers.  Two facts make it parallel:
//   * depth: the left ancestors of leaf i are the strict suffix minima of
//     P_1..P_i and the right ones the strict prefix minima of P_{i+1}..P_{r-1};
//     their powers are distinct, so each side is a bit set over powers, and
//     "drop every power >= p, add p" composes associatively as a pair of
//     masks (A, B): G -> (G & A) | B.  Two scans give every depth (which
//     places each leaf and node in its data array) and M = sum_i depth_i L_i
//     (Sec. 2.3).
//   * ranges: node j of power p merges exactly the leaves whose q share their
//     top p-1 bits with q_j (the level-(p-1) dyadic cell of Method 2'), a
//     contiguous block of the sorted Q array found by galloping search.
#include "common.hpp"
#include "block.hpp"
#include "internal.hpp"

namespace ps {

constexpr int kMaskItems = 16;
constexpr int kMaskBlock = kThreads * kMaskItems;  // 4096 boundaries per block
constexpr uint32_t kNone = 0xFFFFFFFFu;

__device__ __forceinline__ Mask2 mcompose(Mask2 x, Mask2 y) {  // x first, then y
    return Mask2{x.a & y.a, (x.b & y.a) | y.b};
}
__device__ __forceinline__ Mask2 midentity() { return Mask2{~0ull, 0ull}; }
__device__ __forceinline__ Mask2 mof(uint32_t p) {
    return Mask2{p ? ((1ull << p) - 1ull) : 0ull, 1ull << p};
}
__device__ __forceinline__ Mask2 mshfl_up(Mask2 v, int d) {
    return Mask2{__shfl_up(v.a, d), __shfl_up(v.b, d)};
}
__device__ __forceinline__ Mask2 mshfl_down(Mask2 v, int d) {
    return Mask2{__shfl_down(v.a, d), __shfl_down(v.b, d)};
}

// Exclusive forward (left-to-right) scan of thread aggregates over the block.
__device__ __forceinline__ Mask2 block_excl_fwd(Mask2 v, Mask2* sh) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    Mask2 incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        Mask2 o = mshfl_up(incl, d);
        if (lane >= d) incl = mcompose(o, incl);
    }
    Mask2 ex = mshfl_up(incl, 1);
    if (lane == 0) ex = midentity();
    if (lane == 63) sh[wid] = incl;
    __syncthreads();
    Mask2 pre = midentity();
    for (int w2 = 0; w2 < wid; ++w2) pre = mcompose(pre, sh[w2]);
    __syncthreads();
    return mcompose(pre, ex);
}

// Exclusive backward (right-to-left) scan: composition of all threads > tid,
// rightmost first.
__device__ __forceinline__ Mask2 block_excl_bwd(Mask2 v, Mask2* sh) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    Mask2 incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        Mask2 o = mshfl_down(incl, d);
        if (lane + d < 64) incl = mcompose(o, incl);
    }
    Mask2 ex = mshfl_down(incl, 1);
    if (lane == 63) ex = midentity();
    if (lane == 0) sh[wid] = incl;
    __syncthreads();
    Mask2 suf = midentity();
    for (int w2 = kWaves - 1; w2 > wid; --w2) suf = mcompose(suf, sh[w2]);
    __syncthreads();
    return mcompose(suf, ex);
}

__device__ __forceinline__ uint32_t seg_of(const uint64_t* __restrict__ offsets, uint32_t nseg, uint64_t s) {
    // largest g with offsets[g] <= s (the non-empty segment holding s)
    uint32_t lo = 0, hi = nseg + 1;
    while (lo < hi) {
        uint32_t m = (lo + hi) >> 1;
        if (offsets[m] <= s) lo = m + 1; else hi = m;
    }
    return lo - 1;
}

__global__ __launch_bounds__(kThreads) void init_counters_kernel(Counters* c, uint64_t* mc, uint32_t nseg) {
    uint32_t* w = reinterpret_cast<uint32_t*>(c);
    const uint32_t nw = sizeof(Counters) / 4;
    for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < nw; i += gridDim.x * kThreads) w[i] = 0;
    for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < nseg; i += gridDim.x * kThreads) mc[i] = 0;
}

// Fixed-point midpoints Q_i for all leaves.
__global__ __launch_bounds__(kThreads) void leaf_q_kernel(const uint32_t* __restrict__ starts,
                                                           const uint32_t* __restrict__ r_dev,
                                                           const uint64_t* __restrict__ offsets, uint32_t nseg,
                                                           uint64_t* __restrict__ Q) {
    const uint32_t r = *r_dev;
    for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < r; i += gridDim.x * kThreads) {
        const uint32_t s = starts[i], e = starts[i + 1];
        const uint32_t g = seg_of(offsets, nseg, s);
        const uint64_t off = offsets[g], ng = offsets[g + 1] - off;
        const uint64_t twice_mid = (uint64_t)(s - off) + (uint64_t)(e - off);  // 2 (S - off) + L < 2 n
        const uint64_t q = (twice_mid << 32) / (2 * ng);
        Q[i] = ((uint64_t)g << 32) | q;
    }
}

__device__ __forceinline__ uint32_t power_at(const uint64_t* __restrict__ Q, uint32_t j) {
    if (j == 0) return 0;
    const uint64_t x = Q[j - 1] ^ Q[j];
    if (x >> 32) return 0;  // the two leaves lie in different segments
    return (uint32_t)__clz((uint32_t)x) + 1;
}

// Mask scan, phase 1: powers P[j] and per-block forward/backward aggregates.
__global__ __launch_bounds__(kThreads) void mask_reduce_kernel(const uint64_t* __restrict__ Q,
                                                                const uint32_t* __restrict__ r_dev,
                                                                uint8_t* __restrict__ P, Mask2* __restrict__ aggF,
                                                                Mask2* __restrict__ aggB) {
    __shared__ Mask2 sh[kWaves];
    const uint32_t r = *r_dev;
    const uint32_t base = blockIdx.x * kMaskBlock;
    if (base >= r) return;
    Mask2 f = midentity(), b = midentity();
    uint32_t pw[kMaskItems];
#pragma unroll
    for (int i = 0; i < kMaskItems; ++i) {
        const uint32_t j = base + threadIdx.x * kMaskItems + i;
        pw[i] = (j < r) ? power_at(Q, j) : 0;
        if (j < r) {
            P[j] = (uint8_t)pw[i];
            if (j == r - 1) P[r] = 0;
            f = mcompose(f, mof(pw[i]));
        }
    }
#pragma unroll
    for (int i = kMaskItems - 1; i >= 0; --i) {
        const uint32_t j = base + threadIdx.x * kMaskItems + i;
        if (j < r) b = mcompose(b, mof(pw[i]));
    }
    // Block aggregates: forward = threads left to right; backward = right to left.
    Mask2 ef = block_excl_fwd(f, sh);
    Mask2 eb = block_excl_bwd(b, sh);
    if (threadIdx.x == kThreads - 1) aggF[blockIdx.x] = mcompose(ef, f);
    if (threadIdx.x == 0) aggB[blockIdx.x] = mcompose(eb, b);
}

// Mask scan, phase 2 (one block): states entering each block from the left
// (inF) and from the right (inB).
__global__ __launch_bounds__(kThreads) void mask_scan_kernel(const Mask2* __restrict__ aggF,
                                                              const Mask2* __restrict__ aggB,
                                                              const uint32_t* __restrict__ r_dev,
                                                              uint64_t* __restrict__ inF, uint64_t* __restrict__ inB) {
    __shared__ Mask2 sh[kWaves];
    const uint32_t r = *r_dev;
    const uint32_t nb = (r + kMaskBlock - 1) / kMaskBlock;
    const uint32_t per = (nb + kThreads - 1) / kThreads;
    const uint32_t b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
    Mask2 f = midentity(), b = midentity();
    for (uint32_t k = b0; k < b1; ++k) f = mcompose(f, aggF[k]);
    for (uint32_t k = b1; k > b0; --k) b = mcompose(b, aggB[k - 1]);
    Mask2 ef = block_excl_fwd(f, sh);
    Mask2 eb = block_excl_bwd(b, sh);
    Mask2 cf = ef;
    for (uint32_t k = b0; k < b1; ++k) {
        inF[k] = cf.b;
        cf = mcompose(cf, aggF[k]);
    }
    Mask2 cb = eb;
    for (uint32_t k = b1; k > b0; --k) {
        inB[k - 1] = cb.b;
        cb = mcompose(cb, aggB[k - 1]);
    }
}

// Mask scan, phase 3: depths of leaves and nodes, and the merge cost
// M_g = sum over the leaves of segment g of depth * length.
__global__ __launch_bounds__(kThreads) void mask_apply_kernel(const uint8_t* __restrict__ P,
                                                               const uint64_t* __restrict__ Q,
                                                               const uint32_t* __restrict__ starts,
                                                               const uint32_t* __restrict__ r_dev,
                                                               const uint64_t* __restrict__ inF,
                                                               const uint64_t* __restrict__ inB,
                                                               uint8_t* __restrict__ leaf_depth,
                                                               uint8_t* __restrict__ node_depth,
                                                               uint64_t* __restrict__ mc) {
    __shared__ Mask2 sh[kWaves];
    const uint32_t r = *r_dev;
    const uint32_t base = blockIdx.x * kMaskBlock;
    if (base >= r) return;
    const uint32_t j0 = base + threadIdx.x * kMaskItems;
    uint32_t pw[kMaskItems];
    Mask2 f = midentity(), b = midentity();
#pragma unroll
    for (int i = 0; i < kMaskItems; ++i) {
        const uint32_t j = j0 + i;
        pw[i] = (j < r) ? P[j] : 0;
        if (j < r) f = mcompose(f, mof(pw[i]));
    }
#pragma unroll
    for (int i = kMaskItems - 1; i >= 0; --i)
        if (j0 + i < r) b = mcompose(b, mof(pw[i]));
    const Mask2 ef = block_excl_fwd(f, sh);
    const Mask2 eb = block_excl_bwd(b, sh);
    uint64_t G = (inF[blockIdx.x] & ef.a) | ef.b;
    uint64_t Gin[kMaskItems];
#pragma unroll
    for (int i = 0; i < kMaskItems; ++i) {
        Gin[i] = G;
        if (j0 + i < r) {
            const Mask2 m = mof(pw[i]);
            G = (G & m.a) | m.b;
        }
    }
    uint64_t H = (inB[blockIdx.x] & eb.a) | eb.b;
    uint32_t seg_cur = kNone;
    uint64_t acc = 0;
#pragma unroll
    for (int i = kMaskItems - 1; i >= 0; --i) {
        const uint32_t j = j0 + i;
        if (j >= r) continue;
        const Mask2 m = mof(pw[i]);
        const uint64_t Hin = H;
        const uint64_t Gout = (Gin[i] & m.a) | m.b;
        const uint32_t dl = __popcll(Gout >> 1) + __popcll(Hin >> 1);
        leaf_depth[j] = (uint8_t)dl;
        node_depth[j] = (uint8_t)(__popcll((Gin[i] & m.a) >> 1) + __popcll((Hin & m.a) >> 1));
        H = (H & m.a) | m.b;
        const uint32_t g = (uint32_t)(Q[j] >> 32);
        const uint64_t c = (uint64_t)dl * (uint64_t)(starts[j + 1] - starts[j]);
        if (g != seg_cur) {
            if (seg_cur != kNone && acc) atomicAdd((unsigned long long*)&mc[seg_cur], (unsigned long long)acc);
            seg_cur = g;
            acc = 0;
        }
        acc += c;
    }
    // Flush the thread's last partial sum; a wave whose lanes all hold the
    // same segment adds once.
    const int lane = threadIdx.x & 63;
    const uint64_t act = __ballot(seg_cur != kNone);
    const int leader = act ? (__ffsll((unsigned long long)act) - 1) : 0;
    const uint32_t seg0 = __shfl(seg_cur, leader);
    const bool uniform = __all(seg_cur == kNone || seg_cur == seg0);
    if (uniform) {
        uint64_t s = acc;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) s += __shfl_down(s, d);
        if (lane == 0 && act && s) atomicAdd((unsigned long long*)&mc[seg0], (unsigned long long)s);
    } else if (seg_cur != kNone && acc) {
        atomicAdd((unsigned long long*)&mc[seg_cur], (unsigned long long)acc);
    }
}

// Leaf range [Lf, Rt) of every node: the leaves whose Q agree with Q_j on
// the segment and the top P_j - 1 fraction bits.
__global__ __launch_bounds__(kThreads) void node_range_kernel(const uint64_t* __restrict__ Q,
                                                               const uint8_t* __restrict__ P,
                                                               const uint32_t* __restrict__ r_dev,
                                                               const uint32_t* __restrict__ starts,
                                                               uint32_t* __restrict__ Lf, uint32_t* __restrict__ Rt,
                                                               uint32_t* __restrict__ nsize) {
    const uint32_t r = *r_dev;
    for (uint32_t j = blockIdx.x * kThreads + threadIdx.x; j < r; j += gridDim.x * kThreads) {
        const uint32_t p = P[j];
        if (j == 0 || p == 0) continue;
        const uint32_t sh = 33 - p;
        const uint64_t key = Q[j] >> sh;
        // Left: first match in [0, j-1]; Q[j-1] matches.
        int64_t hi = (int64_t)j - 1;
        int64_t d = 1;
        while (hi - d >= 0 && (Q[hi - d] >> sh) == key) d <<= 1;
        int64_t lo = max<int64_t>(0, hi - d + 1), up = hi - (d >> 1);
        while (lo < up) {
            const int64_t m = (lo + up) >> 1;
            if ((Q[m] >> sh) == key) up = m; else lo = m + 1;
        }
        Lf[j] = (uint32_t)lo;
        const uint32_t left = (uint32_t)lo;
        // Right: last match in [j, r-1]; Q[j] matches.
        d = 1;
        while ((int64_t)j + d < (int64_t)r && (Q[j + d] >> sh) == key) d <<= 1;
        lo = (int64_t)j + (d >> 1);
        up = min<int64_t>((int64_t)r - 1, (int64_t)j + d - 1);
        while (lo < up) {
            const int64_t m = (lo + up + 1) >> 1;
            if ((Q[m] >> sh) == key) lo = m; else up = m - 1;
        }
        Rt[j] = (uint32_t)lo + 1;
        nsize[j] = starts[lo + 1] - starts[left];
    }
}

// Appends over the whole block: one atomic per block and counter.
__device__ __forceinline__ uint32_t block_append(bool pred, uint32_t* counter, uint32_t* sh, uint32_t* base_sh) {
    uint32_t total;
    const uint32_t pos = block_excl_sum(pred ? 1u : 0u, sh, &total);
    if (threadIdx.x == 0) *base_sh = total ? atomicAdd(counter, total) : 0u;
    __syncthreads();
    const uint32_t base = *base_sh;
    __syncthreads();
    return pred ? base + pos : kNone;
}

// Classify leaves and nodes: fused-subtree roots (maximal subtrees of at most
// kFuse elements), leaves longer than kFuse, and big nodes (counted per power).
template <int KT>
__global__ __launch_bounds__(kThreads) void classify_kernel(const typename Key<KT>::raw* __restrict__ keys,
                                                             const uint32_t* __restrict__ starts,
                                                             const uint8_t* __restrict__ P,
                                                             const uint32_t* __restrict__ Lf,
                                                             const uint32_t* __restrict__ Rt,
                                                             const uint8_t* __restrict__ leaf_depth,
                                                             const uint8_t* __restrict__ node_depth,
                                                             const uint32_t* __restrict__ nsize,
                                                             Counters* __restrict__ cnt, TreeLists L,
                                                             unsigned long long* __restrict__ prof) {
    using K = Key<KT>;
    constexpr int kIt = 4;  // boundaries per thread per step
    __shared__ uint64_t sh64[kWaves];
    __shared__ uint32_t base_sh[5];
    const uint32_t r = cnt->r;
    auto size_of = [&](uint32_t j) -> uint32_t { return nsize[j]; };
    // profiling element counts, summed per thread and added once per wave
    unsigned long long pr_leaf = 0, pr_fused = 0, pr_merge = 0;
    for (uint32_t i0 = blockIdx.x * kThreads * kIt; i0 < r; i0 += gridDim.x * kThreads * kIt) {
        // flags of node i and leaf i for this thread's kIt indices; the five
        // lists (big nodes, the three kinds of units, big leaves) take slots
        // from one packed block scan (12-bit fields) and one atomic per list
        // per step
        uint8_t fl[kIt];
        uint8_t mode[kIt];
        uint8_t kn[kIt], kl[kIt];  // kinds of the unit node and unit leaf
        uint32_t nlf[kIt], nrt[kIt];
        uint64_t mine = 0;
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const uint32_t i = i0 + it * kThreads + threadIdx.x;
            const bool valid = i < r;
            uint8_t f = 0;
            mode[it] = kLeafNoop;
            kn[it] = kl[it] = 0;
            nlf[it] = nrt[it] = 0;
            // ---- node i (boundary between leaves i-1 and i)
            if (valid && i >= 1 && P[i] >= 1) {
                nlf[it] = Lf[i];
                nrt[it] = Rt[i];
                // the parent is the nearer of the two bounding boundaries,
                // the one with the larger power (two ancestors never share
                // a power; both 0 only at a segment root)
                const uint32_t pl = P[nlf[it]], pr = P[nrt[it]];
                const uint32_t par = pl > pr ? nlf[it] : (pr > pl ? nrt[it] : kNone);
                if (par == nrt[it]) L.child_l[par] = i;
                else if (par != kNone) L.child_r[par] = i;
                const uint32_t sz = nsize[i];
                if (sz > (uint32_t)kFuse) {
                    // a merge of its own pass, unless two-level passes absorb
                    // it into its parent (big nodes at odd depth)
                    if (L.levels != 2 || (node_depth[i] & 1u) == 0) {
                        f |= 1;
                        pr_merge += sz;
                        // does it absorb a child: one of more than kFuse
                        // elements that is not a single leaf
                        if (L.levels == 2) {
                            const uint32_t s0 = starts[nlf[it]], sm = starts[i], s1 = starts[nrt[it]];
                            if ((nlf[it] + 1 < i && sm - s0 > (uint32_t)kFuse) ||
                                (i + 1 < nrt[it] && s1 - sm > (uint32_t)kFuse))
                                f |= 16;
                        }
                    }
                } else if ((par == kNone) || size_of(par) > (uint32_t)kFuse) {
                    f |= 2;  // unit node
                    kn[it] = (uint8_t)unit_kind(sizeof(typename K::ukey), nrt[it] - nlf[it], sz);
                }
            }
            // ---- leaf i
            if (valid) {
                const uint32_t s = starts[i], len = starts[i + 1] - s;
                const uint32_t pl = P[i], pr = P[i + 1];
                const uint32_t par = pl > pr ? i : (pr > pl ? i + 1 : kNone);
                if (len > (uint32_t)kFuse) {
                    f |= 8;  // big leaf
                    const bool desc = K::ord(keys[s + 1]) < K::ord(keys[s]);
                    const bool moved = big_leaf_buf(pass_level(leaf_depth[i], L.levels), L.nbuf) != 0;
                    mode[it] = desc ? (moved ? kLeafRevCopy : kLeafRevInPlace) : (moved ? kLeafCopy : kLeafNoop);
                } else if ((par == kNone) || size_of(par) > (uint32_t)kFuse) {
                    f |= 4;  // unit leaf
                    kl[it] = (uint8_t)unit_kind(sizeof(typename K::ukey), 1, len);
                }
            }
            fl[it] = f;
            // fields: big nodes, units of kind 0, 1, 2, big leaves (each
            // count <= kThreads * kIt < 2^12)
            mine += (uint64_t)(f & 1) + ((uint64_t)((f >> 3) & 1) << 48);
            if (f & 2) mine += 1ull << (12 * (1 + kn[it]));
            if (f & 4) mine += 1ull << (12 * (1 + kl[it]));
        }
        static_assert(kThreads * kIt < (1 << 12), "block counts fit 12-bit fields");
        uint64_t total;
        uint64_t off = block_excl_sum64(mine, sh64, &total);
        if (threadIdx.x < 5) {
            const uint32_t c = (uint32_t)(total >> (12 * threadIdx.x)) & 0xFFFu;
            uint32_t* ctr = threadIdx.x == 0 ? &cnt->nbig : threadIdx.x == 4 ? &cnt->nbigleaf
                                                         : &cnt->nunit[threadIdx.x - 1];
            base_sh[threadIdx.x] = c ? atomicAdd(ctr, c) : 0u;
        }
        __syncthreads();
        uint32_t pos[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) pos[q] = base_sh[q] + ((uint32_t)(off >> (12 * q)) & 0xFFFu);
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const uint32_t i = i0 + it * kThreads + threadIdx.x;
            const uint8_t f = fl[it];
            if (f & 1) L.biglist[pos[0]++] = i | ((f & 16) ? 0x80000000u : 0u);
            if (f & 2) {
                const uint32_t slot = L.unit_base[kn[it]] + pos[1 + kn[it]]++;
                pr_fused += starts[nrt[it]] - starts[nlf[it]];
                L.unit_rec[slot] = UnitRec{nlf[it], nrt[it], starts[nlf[it]], starts[nrt[it]]};
                L.unit_par[slot] = node_buf(pass_level(node_depth[i], L.levels), L.nbuf);
            }
            if (f & 4) {
                const uint32_t slot = L.unit_base[kl[it]] + pos[1 + kl[it]]++;
                pr_fused += starts[i + 1] - starts[i];
                L.unit_rec[slot] = UnitRec{i, i + 1, starts[i], starts[i + 1]};
                L.unit_par[slot] = node_buf(pass_level(leaf_depth[i], L.levels), L.nbuf);
            }
            if (f & 8) {
                const uint32_t slot = pos[4]++;
                if (mode[it] != kLeafNoop) pr_leaf += starts[i + 1] - starts[i];
                L.bigleaf[slot] = i;
                L.bigleaf_mode[slot] = mode[it];
            }
        }
    }
    if (prof) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            pr_leaf += __shfl_xor(pr_leaf, o);
            pr_fused += __shfl_xor(pr_fused, o);
            pr_merge += __shfl_xor(pr_merge, o);
        }
        if ((threadIdx.x & 63) == 0) {
            if (pr_leaf) atomicAdd(&prof[3], pr_leaf);
            if (pr_fused) atomicAdd(&prof[4], pr_fused);
            if (pr_merge) atomicAdd(&prof[5], pr_merge);
        }
    }
}

// Adds 1 per active lane to counter[key], one atomic per distinct key in
// the wave; returns the lane's slot among those lanes (ordered by lane).
__device__ __forceinline__ uint32_t wave_count_by_key(bool active, uint32_t key, uint32_t* counter) {
    const int lane = threadIdx.x & 63;
    uint32_t slot = kNone;
    bool done = !active;
    while (true) {
        const uint64_t act = __ballot(!done);
        if (!act) break;
        const int leader = __ffsll((unsigned long long)act) - 1;
        const uint32_t kl = __shfl(key, leader);
        const uint64_t same = __ballot(!done && key == kl);
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&counter[kl], (uint32_t)__popcll(same));
        base = __shfl(base, leader);
        if (!done && key == kl) {
            slot = base + (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
            done = true;
        }
    }
    return slot;
}

// The bucket key of a big-node list entry: 2 p + 1 for a node of power p
// that absorbs a child, 2 p otherwise.  Within its power's bucket a node that
// absorbs a child comes after every node that does not.
__device__ __forceinline__ uint32_t bucket_key(const uint8_t* __restrict__ P, uint32_t e) {
    return 2u * P[e & 0x7FFFFFFFu] + (e >> 31);
}
constexpr int kKeys = 2 * (kMaxPass + 1);

// Big nodes per power (and how many absorb a child): counted per block in
// LDS, then one atomic per key per block (a few dozen global counters take
// every update).
__global__ __launch_bounds__(kThreads) void bucket_count_kernel(const uint8_t* __restrict__ P,
                                                                 Counters* __restrict__ cnt, TreeLists L) {
    __shared__ uint32_t h[kKeys];
    const uint32_t nbig = cnt->nbig;
    for (uint32_t i = threadIdx.x; i < (uint32_t)kKeys; i += kThreads) h[i] = 0;
    __syncthreads();
    for (uint32_t k0 = blockIdx.x * kThreads; k0 < nbig; k0 += gridDim.x * kThreads) {
        const uint32_t k = k0 + threadIdx.x;
        const bool valid = k < nbig;
        wave_count_by_key(valid, valid ? bucket_key(P, L.biglist[k]) : 0u, h);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < (uint32_t)kKeys; i += kThreads) {
        if (!h[i]) continue;
        atomicAdd(&cnt->pcount[i >> 1], h[i]);
        if (i & 1u) atomicAdd(&cnt->pcount_q[i >> 1], h[i]);
    }
}

__global__ void bucket_base_kernel(Counters* cnt) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        uint32_t acc = 0;
        for (int p = 0; p <= kMaxPass; ++p) {
            cnt->pbase[p] = acc;
            cnt->pfill[p] = 0;
            cnt->pqfill[p] = 0;
            acc += cnt->pcount[p];
        }
    }
}

// Each block counts its nodes per key in LDS, reserves that many slots of
// every bucket with one atomic per key (nodes that absorb a child from the
// bucket's tail part), then hands them out in LDS.
__global__ __launch_bounds__(kThreads) void bucket_scatter_kernel(const uint8_t* __restrict__ P,
                                                                   Counters* __restrict__ cnt, TreeLists L) {
    __shared__ uint32_t h[kKeys];
    const uint32_t nbig = cnt->nbig;
    for (uint32_t i = threadIdx.x; i < (uint32_t)kKeys; i += kThreads) h[i] = 0;
    __syncthreads();
    for (uint32_t k0 = blockIdx.x * kThreads; k0 < nbig; k0 += gridDim.x * kThreads) {
        const uint32_t k = k0 + threadIdx.x;
        const bool valid = k < nbig;
        wave_count_by_key(valid, valid ? bucket_key(P, L.biglist[k]) : 0u, h);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < (uint32_t)kKeys; i += kThreads) {
        if (!h[i]) continue;
        const uint32_t p = i >> 1;
        h[i] = (i & 1u) ? cnt->pbase[p] + (cnt->pcount[p] - cnt->pcount_q[p]) + atomicAdd(&cnt->pqfill[p], h[i])
                        : cnt->pbase[p] + atomicAdd(&cnt->pfill[p], h[i]);
    }
    __syncthreads();
    // h[key] is now the block's next free slot of that part of its bucket
    for (uint32_t k0 = blockIdx.x * kThreads; k0 < nbig; k0 += gridDim.x * kThreads) {
        const uint32_t k = k0 + threadIdx.x;
        const bool valid = k < nbig;
        const uint32_t e = valid ? L.biglist[k] : 0;
        const uint32_t slot = wave_count_by_key(valid, valid ? bucket_key(P, e) : 0u, h);
        if (valid) L.bucket[slot] = e & 0x7FFFFFFFu;
    }
}

// Tile prefix of each power bucket (block p >= 1) and of the big leaves (block 0).
__global__ __launch_bounds__(kThreads) void tile_scan_kernel(const uint32_t* __restrict__ starts,
                                                              const uint32_t* __restrict__ Lf,
                                                              const uint32_t* __restrict__ Rt,
                                                              const uint8_t* __restrict__ node_depth,
                                                              Counters* __restrict__ cnt, TreeLists L,
                                                              uint32_t merge_tile) {
    __shared__ uint32_t sh[kWaves];
    constexpr int kIt = 8;  // entries per thread per step, in position order
    const uint32_t p = blockIdx.x;
    const uint32_t n = (p == 0) ? cnt->nbigleaf : cnt->pcount[p];
    const uint32_t off = (p == 0) ? 0 : cnt->pbase[p];
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < n; c0 += kThreads * kIt) {
        // all of a step's loads are independent, so they overlap
        uint32_t tiles[kIt];
        uint32_t sum = 0;
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const uint32_t k = c0 + threadIdx.x * kIt + it;
            tiles[it] = 0;
            if (k >= n) continue;
            if (p == 0) {
                const uint32_t i = L.bigleaf[k];
                const uint32_t len = starts[i + 1] - starts[i];
                const uint8_t mode = L.bigleaf_mode[k];
                if (mode == kLeafRevInPlace) tiles[it] = (len / 2 + kLeafTile - 1) / kLeafTile;
                else if (mode != kLeafNoop) tiles[it] = (len + kLeafTile - 1) / kLeafTile;
            } else {
                const uint32_t j = L.bucket[off + k];
                const uint32_t lf = Lf[j], rt = Rt[j];
                const uint32_t lo = starts[lf], mid = starts[j], hi = starts[rt];
                const uint32_t d = node_depth[j];
                // An input of the merge that is one leaf longer than a fused
                // subtree is in the long-leaf array; any other input is a
                // node or a fused subtree, in its pass level's array.
                auto in_buf = [&](bool one_leaf, uint32_t size, uint32_t depth) -> uint32_t {
                    const uint32_t lv = pass_level(depth, L.levels);
                    return (one_leaf && size > (uint32_t)kFuse) ? big_leaf_buf(lv, L.nbuf) : node_buf(lv, L.nbuf);
                };
                // A child of more than kFuse elements that is not one leaf is
                // a big node; at odd depth, with two-level passes, it is
                // merged here: its children are the inputs.
                uint32_t m1 = mid, m2 = hi, ba, bb = 0, bc, bd = 0;
                // (a child index outside the node's leaves would mean
                // inconsistent lists: the child is then taken as an input,
                // which keeps every access inside the node)
                const uint32_t kl = (L.levels == 2 && lf + 1 < j) ? L.child_l[j] : 0u;
                const uint32_t kr = (L.levels == 2 && j + 1 < rt) ? L.child_r[j] : 0u;
                if (L.levels == 2 && lf + 1 < j && mid - lo > (uint32_t)kFuse && kl > lf && kl < j) {
                    m1 = starts[kl];
                    ba = in_buf(lf + 1 == kl, m1 - lo, d + 2);
                    bb = in_buf(kl + 1 == j, mid - m1, d + 2);
                } else {
                    ba = in_buf(lf + 1 == j, mid - lo, d + 1);
                }
                if (L.levels == 2 && j + 1 < rt && hi - mid > (uint32_t)kFuse && kr > j && kr < rt) {
                    m2 = starts[kr];
                    bc = in_buf(j + 1 == kr, m2 - mid, d + 2);
                    bd = in_buf(kr + 1 == rt, hi - m2, d + 2);
                } else {
                    bc = in_buf(j + 1 == rt, hi - mid, d + 1);
                }
                const NodeRec R{lo, m1, mid, m2, hi,
                                node_buf(pass_level(d, L.levels), L.nbuf) | (ba << 2) | (bb << 4) | (bc << 6) |
                                    (bd << 8)};
                L.node_rec[off + k] = R;
                if (node_is_quad(R)) {
                    // boundaries every kQuadSpacing along each child's merge,
                    // plus the start
                    const uint32_t g = kQuadSpacing;
                    tiles[it] = (mid - lo - 1) / g + (hi - mid - 1) / g + 1;
                } else {
                    tiles[it] = (hi - lo + merge_tile - 1) / merge_tile;
                }
            }
            sum += tiles[it];
        }
        uint32_t total;
        uint32_t run = carry + block_excl_sum(sum, sh, &total);
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const uint32_t k = c0 + threadIdx.x * kIt + it;
            if (k < n) {
                if (p == 0) L.leaf_tile[k] = run;
                else L.bucket_tile[off + k] = run;
                // the first node that absorbs a child starts the pass's second part
                if (p > 0 && k == n - cnt->pcount_q[p]) cnt->ptq[p] = run;
            }
            run += tiles[it];
        }
        carry += total;
    }
    if (threadIdx.x == 0) {
        cnt->ptiles[p] = carry;
        if (p > 0 && cnt->pcount_q[p] == 0) cnt->ptq[p] = carry;
    }
}

// First split record of every pass.
__global__ void pass_base_kernel(Counters* cnt) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        uint32_t acc = 0;
        for (int p = 1; p <= kMaxPass; ++p) {
            cnt->sbase[p] = acc;
            acc += cnt->ptiles[p];
        }
        cnt->sbase[0] = acc;
    }
}

// ------------------------------------------------------------------ peeksort
//
// Alg. PeekSort (Sec. 3.1) builds the tree top-down: a range of whole leaves
// A[l..r] (first leaf A[l..e], last leaf A[s..r]) with m = l + floor((r-l)/2)
// is cut after its first leaf if m <= e, before its last leaf if m >= s, and
// otherwise at the nearer end of the leaf A[i..j] containing m: before it if
// m - i < j - m, else after it.  One launch per two depths: the launch for
// depth d reads the ranges of depth d, writes the nodes of depths d and
// d + 1 and the ranges of depth d + 2.  Node j (the cut of a range at depth
// t, between leaves j-1 and j) gets the merge-pass key P[j] = t + 1, so
// children (deeper) merge before their parent, exactly as with node powers;
// boundaries that are not nodes keep P = 0.

// lower_bound over starts[0..n): first k with starts[k] >= v.
__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t* __restrict__ a, uint32_t n, uint64_t v) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t m = (lo + hi) >> 1;
        if ((uint64_t)a[m] < v) lo = m + 1; else hi = m;
    }
    return lo;
}

// Per segment: its leaves, the root range (two or more leaves) or the
// depth-0 single leaf, and P = 0 at the segment's first boundary.
__global__ __launch_bounds__(kThreads) void peek_roots_kernel(const uint32_t* __restrict__ starts,
                                                              const uint64_t* __restrict__ offsets, uint32_t nseg,
                                                              Counters* __restrict__ cnt, PeekRange* __restrict__ F0,
                                                              uint32_t cap, uint8_t* __restrict__ P,
                                                              uint8_t* __restrict__ leaf_depth) {
    __shared__ uint32_t sh[kWaves];
    __shared__ uint32_t base_sh;
    const uint32_t r = cnt->r;
    if (blockIdx.x == 0 && threadIdx.x == 0) P[r] = 0;
    for (uint32_t g0 = blockIdx.x * kThreads; g0 < nseg; g0 += gridDim.x * kThreads) {
        const uint32_t g = g0 + threadIdx.x;
        uint32_t a = 0, b = 0;
        if (g < nseg) {
            a = lower_bound_u32(starts, r + 1, offsets[g]);
            b = lower_bound_u32(starts, r + 1, offsets[g + 1]);
            if (b > r) b = r;
            if (a < b) P[a] = 0;
            if (b - a == 1) leaf_depth[a] = 0;
        }
        const bool root = g < nseg && b >= a + 2;
        const uint32_t slot = block_append(root, &cnt->peek_count[0], sh, &base_sh);
        if (root && slot < cap) F0[slot] = PeekRange{a, b, g, 0};
    }
}

// The cut of a range of whole leaves [a, b), b - a >= 2 (Alg. PeekSort).
__device__ __forceinline__ uint32_t peek_cut(const uint32_t* __restrict__ starts, uint32_t a, uint32_t b) {
    const uint32_t l = starts[a], r = starts[b] - 1;
    const uint32_t e = starts[a + 1] - 1, s = starts[b - 1];
    const uint32_t m = l + (r - l) / 2;
    if (m <= e) return a + 1;
    if (m >= s) return b - 1;
    // leaf kk of (a, b) with starts[kk] <= m < starts[kk+1]
    uint32_t lo = a, hi = b;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (starts[mid] <= m) lo = mid; else hi = mid;
    }
    const uint32_t i = starts[lo], j = starts[lo + 1] - 1;
    return (m - i < j - m) ? lo : lo + 1;
}

// Two depths per launch: each range of depth d is cut, then each of its
// parts with two or more leaves (depth d + 1, if that depth can hold a node)
// is cut as well, and the parts of those with two or more leaves are the
// ranges of depth d + 2.  Node j = cut of a range at depth t gets P[j] =
// t + 1, its depth, its leaf range and size; a part of one leaf gets its
// leaf depth.  Halves the dependent launches of the level-by-level build.
__global__ __launch_bounds__(kThreads) void peek_level_kernel(const uint32_t* __restrict__ starts,
                                                              Counters* __restrict__ cnt,
                                                              const PeekRange* __restrict__ Fin,
                                                              PeekRange* __restrict__ Fout, uint32_t cap,
                                                              uint32_t d, uint32_t levels, uint8_t* __restrict__ P,
                                                              uint8_t* __restrict__ node_depth,
                                                              uint8_t* __restrict__ leaf_depth,
                                                              uint32_t* __restrict__ Lf, uint32_t* __restrict__ Rt,
                                                              uint32_t* __restrict__ nsize,
                                                              unsigned long long* __restrict__ mc) {
    __shared__ uint32_t sh[kWaves];
    __shared__ uint32_t base_sh;
    const uint32_t nin = min(cnt->peek_count[d], cap);
    // records node `cut` of the range [a, b) at depth t; returns its size
    auto node = [&](uint32_t a, uint32_t b, uint32_t cut, uint32_t t) {
        const uint32_t size = starts[b] - starts[a];
        P[cut] = (uint8_t)(t + 1);
        node_depth[cut] = (uint8_t)t;
        Lf[cut] = a;
        Rt[cut] = b;
        nsize[cut] = size;
        if (cut - a == 1) leaf_depth[a] = (uint8_t)(t + 1);
        if (b - cut == 1) leaf_depth[cut] = (uint8_t)(t + 1);
        return size;
    };
    for (uint32_t k0 = blockIdx.x * kThreads; k0 < nin; k0 += gridDim.x * kThreads) {
        const uint32_t k = k0 + threadIdx.x;
        const bool valid = k < nin;
        uint32_t g = 0, size = 0, nout = 0;
        uint32_t oa[4], ob[4];
        if (valid) {
            const PeekRange R = Fin[k];
            g = R.g;
            const uint32_t cut = peek_cut(starts, R.a, R.b);
            size = node(R.a, R.b, cut, d);
            const uint32_t pa[2] = {R.a, cut}, pb[2] = {cut, R.b};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (pb[h] - pa[h] >= 2 && d + 1 < levels) {
                    const uint32_t c2 = peek_cut(starts, pa[h], pb[h]);
                    size += node(pa[h], pb[h], c2, d + 1);
                    if (c2 - pa[h] >= 2) {
                        oa[nout] = pa[h];
                        ob[nout++] = c2;
                    }
                    if (pb[h] - c2 >= 2) {
                        oa[nout] = c2;
                        ob[nout++] = pb[h];
                    }
                }
            }
        }
        // M = sum of merge result sizes, per segment: one atomic per wave for
        // the lanes of the first active lane's segment, one per other lane
        {
            const uint64_t act = __ballot(valid);
            if (act) {
                const int leader = __ffsll((unsigned long long)act) - 1;
                const uint32_t gl = __shfl(g, leader);
                const bool same = valid && g == gl;
                unsigned long long v = same ? (unsigned long long)size : 0ull;
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
                if ((int)(threadIdx.x & 63) == leader) atomicAdd(&mc[gl], v);
                if (valid && !same) atomicAdd(&mc[g], (unsigned long long)size);
            }
        }
        uint32_t total;
        const uint32_t pos = block_excl_sum(nout, sh, &total);
        if (threadIdx.x == 0) base_sh = total ? atomicAdd(&cnt->peek_count[d + 2], total) : 0u;
        __syncthreads();
        const uint32_t base = base_sh + pos;
        __syncthreads();
        for (uint32_t q = 0; q < nout; ++q)
            if (base + q < cap) Fout[base + q] = PeekRange{oa[q], ob[q], g, 0};
    }
}

// ------------------------------------------------------------- host launch

static inline uint32_t grid_for(uint64_t items, uint32_t cap) {
    uint64_t g = (items + kThreads - 1) / kThreads;
    if (g < 1) g = 1;
    return (uint32_t)(g < cap ? g : cap);
}

hipError_t launch_init(Counters* cnt, uint64_t* mc, uint32_t nseg, hipStream_t st) {
    hipLaunchKernelGGL(init_counters_kernel, dim3(grid_for(nseg + 64, 1024)), dim3(kThreads), 0, st, cnt, mc, nseg);
    return hipGetLastError();
}

// Powers, depths and merge cost (everything ps_merge_cost needs).
hipError_t launch_tree_cost(const TreeArgs& a, hipStream_t st) {
    const uint32_t* r_dev = &a.cnt->r;
    const uint32_t gl = grid_for(a.rmax, 4096);
    hipLaunchKernelGGL(leaf_q_kernel, dim3(gl), dim3(kThreads), 0, st, a.starts, r_dev, a.offsets, a.nseg, a.Q);
    const uint32_t nb = (a.rmax + kMaskBlock - 1) / kMaskBlock;
    hipLaunchKernelGGL(mask_reduce_kernel, dim3(nb), dim3(kThreads), 0, st, a.Q, r_dev, a.P, a.aggF, a.aggB);
    hipLaunchKernelGGL(mask_scan_kernel, dim3(1), dim3(kThreads), 0, st, a.aggF, a.aggB, r_dev, a.inF, a.inB);
    hipLaunchKernelGGL(mask_apply_kernel, dim3(nb), dim3(kThreads), 0, st, a.P, a.Q, a.starts, r_dev, a.inF, a.inB,
                       a.leaf_depth, a.node_depth, a.mc);
    return hipGetLastError();
}

template <int KT>
static void launch_classify_t(const TreeArgs& a, uint32_t g, hipStream_t st) {
    using raw = typename Key<KT>::raw;
    hipLaunchKernelGGL(classify_kernel<KT>, dim3(g), dim3(kThreads), 0, st, (const raw*)a.keys, a.starts, a.P, a.Lf,
                       a.Rt, a.leaf_depth, a.node_depth, a.nsize, a.cnt, a.lists, a.prof);
}

// Node ranges and the work lists of the data-movement phase.
hipError_t launch_node_ranges(const TreeArgs& a, hipStream_t st) {
    const uint32_t gl = grid_for(a.rmax, 4096);
    hipLaunchKernelGGL(node_range_kernel, dim3(gl), dim3(kThreads), 0, st, a.Q, a.P, &a.cnt->r, a.starts, a.Lf, a.Rt,
                       a.nsize);
    return hipGetLastError();
}

hipError_t launch_tree_lists(int kt, const TreeArgs& a, hipStream_t st) {
    // fewer blocks: each step of a block is one atomic per list on a shared counter
    const uint32_t gl = grid_for((a.rmax + 3) / 4, 1024);
    switch (kt) {
    case KT_I32: launch_classify_t<KT_I32>(a, gl, st); break;
    case KT_U32: launch_classify_t<KT_U32>(a, gl, st); break;
    case KT_I64: launch_classify_t<KT_I64>(a, gl, st); break;
    case KT_U64: launch_classify_t<KT_U64>(a, gl, st); break;
    case KT_F32: launch_classify_t<KT_F32>(a, gl, st); break;
    default: return hipErrorInvalidValue;
    }
    const uint32_t gb = grid_for(a.rmax, 512);
    hipLaunchKernelGGL(bucket_count_kernel, dim3(gb), dim3(kThreads), 0, st, a.P, a.cnt, a.lists);
    hipLaunchKernelGGL(bucket_base_kernel, dim3(1), dim3(64), 0, st, a.cnt);
    hipLaunchKernelGGL(bucket_scatter_kernel, dim3(gb), dim3(kThreads), 0, st, a.P, a.cnt, a.lists);
    hipLaunchKernelGGL(tile_scan_kernel, dim3(kMaxPass + 1), dim3(kThreads), 0, st, a.starts, a.Lf, a.Rt,
                       a.node_depth, a.cnt, a.lists, a.merge_tile);
    hipLaunchKernelGGL(pass_base_kernel, dim3(1), dim3(64), 0, st, a.cnt);
    return hipGetLastError();
}

hipError_t launch_peek_tree(const TreeArgs& a, PeekRange* f0, PeekRange* f1, uint32_t cap, uint32_t levels,
                            hipStream_t st) {
    hipLaunchKernelGGL(peek_roots_kernel, dim3(grid_for(a.nseg, 1024)), dim3(kThreads), 0, st, a.starts, a.offsets,
                       a.nseg, a.cnt, f0, cap, a.P, a.leaf_depth);
    const uint32_t g = grid_for(cap, 2048);
    for (uint32_t d = 0; d < levels; d += 2) {
        PeekRange* fin = (d & 2) ? f1 : f0;
        PeekRange* fout = (d & 2) ? f0 : f1;
        hipLaunchKernelGGL(peek_level_kernel, dim3(g), dim3(kThreads), 0, st, a.starts, a.cnt, fin, fout, cap, d,
                           levels, a.P, a.node_depth, a.leaf_depth, a.Lf, a.Rt, a.nsize, (unsigned long long*)a.mc);
    }
    return hipGetLastError();
}

}  // namespace ps
