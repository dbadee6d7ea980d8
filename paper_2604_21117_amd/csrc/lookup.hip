// Lookup and range batches.
//
// Lookup (paper Sections IV-A, IV-E, IV-F): every query descends from the
// root with a group of G lanes (see traverse.h), the top inner levels read
// from the LDS copy of the mirror, the rest from HBM; at the leaf an
// equality ballot over the key line gives the slot, and one lane reads the
// value.  A key that is not found returns all ones with found = 0 (the
// paper's -1 result, Section IV-D).  Results go to the caller's order.
//
// Range (an addition over the linked leaves of Section III): the
// group descends to the leaf of `lo`, then walks the leaf chain; per leaf a
// ballot marks the slots with lo <= key <= hi and the group writes them in
// slot order at out[offset + running count], until `max` pairs are written,
// a key above `hi` is seen or the chain ends.
//
// Both kernels are persistent: a grid of at most a few thousand
// workgroups walks tiles of queries, so the mirror is staged once per
// workgroup.
#include "common.h"
#include "traverse.h"
#include "kernels.h"

namespace gt {

constexpr int kLookupBlock = 256;

// Leaf stage shared by the lookup kernels: match the key line, take the
// value (from the co-loaded value line, or by one dependent read), write the
// result of every live query.  NT selects non-temporal loads: bit 0 the key
// line, bit 1 the value line (a lookup reads a value line once, so
// streaming it keeps the lines that are reused -- leaf parents, upper
// levels -- in L2).
template <class K, int G, int QPG, bool VC, int NT>
__device__ __forceinline__ void finish_lookups(const TreeView<K>& t, const K (&key)[QPG], const uint32_t (&leaf)[QPG],
                                               const uint64_t (&qi)[QPG], bool empty, int gl, int gbase,
                                               K* __restrict__ vout, uint8_t* __restrict__ fout) {
    using T = Trav<K, G>;
    typename T::KV kv[QPG];
    typename T::KV vv[QPG];
#pragma unroll
    for (int j = 0; j < QPG; ++j) {
        const K* kl = t.lkeys + static_cast<uint64_t>(leaf[j]) * kSlots;
        const K* vl = t.lvals + static_cast<uint64_t>(leaf[j]) * kSlots;
        if constexpr ((NT & 1) != 0) kv[j] = T::load_keys_nt(kl, gl);
        else kv[j] = T::load_keys(kl, gl);
        if constexpr (VC) {
            if constexpr ((NT & 2) != 0) vv[j] = T::load_keys_nt(vl, gl);
            else vv[j] = T::load_keys(vl, gl);
        }
    }
    uint32_t slot[QPG];
#pragma unroll
    for (int j = 0; j < QPG; ++j) slot[j] = T::match_slot(kv[j], key[j], gbase);
    K val[QPG];
    bool hit[QPG];
#pragma unroll
    for (int j = 0; j < QPG; ++j) {
        hit[j] = slot[j] < kSlots && !empty;
        val[j] = kmax<K>();
        if constexpr (VC) {
            const K x = T::pick_value(vv[j], hit[j] ? slot[j] : 0u, gbase);
            if (hit[j]) val[j] = x;
        } else {
            if (gl == (j % G) && qi[j] != ~0ull && hit[j]) {
                const K* vp = t.lvals + static_cast<uint64_t>(leaf[j]) * kSlots + slot[j];
                if constexpr ((NT & 2) != 0) val[j] = __builtin_nontemporal_load(vp);
                else val[j] = *vp;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < QPG; ++j) {
        if (gl == (j % G) && qi[j] != ~0ull) {
            vout[qi[j]] = val[j];
            fout[qi[j]] = hit[j] ? 1 : 0;
        }
    }
}

template <class K, int G, int QPG, int LV, bool VC, int NT>
__global__ __launch_bounds__(kLookupBlock) void k_lookup(TreeView<K> t, const K* __restrict__ q, uint64_t B,
                                                          K* __restrict__ vout, uint8_t* __restrict__ fout,
                                                          uint64_t ntiles) {
    extern __shared__ __align__(16) uint8_t lds[];
    const uint8_t* mir = t.mirror;
    uint32_t mnodes = kMirrorMaxNodes;
    if constexpr (LV > 0) {
        mnodes = mirror_nodes_for_levels(LV);
        stage_mirror<K>(t.mirror, lds, mnodes);
        __syncthreads();
        mir = lds;
    }
    const MirrorHeader* mh = reinterpret_cast<const MirrorHeader*>(mir);
    const bool empty = mh->n_keys == 0;
    const int lane = lane_id();
    const int gl = lane % G, gbase = lane - gl;
    const uint64_t group = threadIdx.x / G;
    const uint64_t tile_q = static_cast<uint64_t>(kLookupBlock / G) * QPG;
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        K key[QPG];
        uint64_t qi[QPG];
#pragma unroll
        for (int j = 0; j < QPG; ++j) {
            const uint64_t x = tile * tile_q + group * QPG + j;
            key[j] = x < B ? q[x] : K(0);
            qi[j] = x < B ? x : ~0ull;
        }
        uint32_t leaf[QPG];
        descend<K, G, QPG, false>(t, mir, mnodes, LV, key, leaf, gl, gbase);
        finish_lookups<K, G, QPG, VC, NT>(t, key, leaf, qi, empty, gl, gbase, vout, fout);
    }
}

// Position of the t-th set bit (t counted from 0) of m; m has more than t.
__device__ __forceinline__ int nth_set_bit(uint64_t m, uint32_t t) {
    int pos = 0;
#pragma unroll
    for (int w = 32; w > 0; w >>= 1) {
        const uint32_t c = static_cast<uint32_t>(__popcll(m & ((1ull << w) - 1ull)));
        if (t >= c) {
            t -= c;
            m >>= w;
            pos += w;
        }
    }
    return pos;
}

// XCD-split lookup for large batches.  The dispatcher deals the workgroups
// of a launch to the eight XCDs in turn, so workgroups w and w + 8 share an
// XCD and its L2 (which XCD takes workgroup 0 varies; only the grouping is
// used).  Seven splitter keys cut the key space into eight ranges, and the
// workgroups with w % 8 == x answer the queries of range x only, so the leaf
// parents they read (an eighth of them) stay in one L2.  Every wave of group
// x reads four 64-query chunks of the batch at a time (one coalesced load
// each), keeps the queries of its range with one ballot per chunk, and deals
// them to its eight 8-lane groups, four queries per group per round.  Each
// chunk is read by one wave of every XCD; results go by
// query index, so the output is the plain kernel's.  All lanes stay active
// through a round (the groups' cross-lane reads need their source lanes).
constexpr int kXcdChunks = 4;  // 64-query chunks a wave reads at once

template <class K, bool VC, int NT>
__global__ __launch_bounds__(kLookupBlock) void k_lookup_xcd(TreeView<K> t, const K* __restrict__ q, uint64_t B,
                                                              K* __restrict__ vout, uint8_t* __restrict__ fout,
                                                              uint64_t nchunks) {
    constexpr int G = 8, LV = 2, QPG = kXcdChunks;
    constexpr uint32_t kGroups = 64 / G;
    extern __shared__ __align__(16) uint8_t lds[];
    const uint32_t mnodes = mirror_nodes_for_levels(LV);
    stage_mirror<K>(t.mirror, lds, mnodes);
    const MirrorHeader* gmh = reinterpret_cast<const MirrorHeader*>(t.mirror);
    const K* sp = reinterpret_cast<const K*>(t.mirror + MirrorLayout<K>::split_off());
    const uint32_t nsplit = gmh->nsplit;
    K split[kXcds - 1];
#pragma unroll
    for (int x = 0; x < kXcds - 1; ++x) split[x] = sp[x];
    __syncthreads();
    const bool empty = reinterpret_cast<const MirrorHeader*>(lds)->n_keys == 0;
    const uint32_t xcd = blockIdx.x % kXcds;
    const int lane = lane_id();
    const int gl = lane % G, gbase = lane - gl;
    const uint32_t grp = static_cast<uint32_t>(lane / G);
    constexpr int kWaves = kLookupBlock / 64;
    const uint64_t wave_in_xcd = static_cast<uint64_t>(blockIdx.x / kXcds) * kWaves + threadIdx.x / 64;
    const uint64_t waves_per_xcd = static_cast<uint64_t>(gridDim.x / kXcds) * kWaves;
    const uint64_t nsets = (nchunks + kXcdChunks - 1) / kXcdChunks;
    for (uint64_t set = wave_in_xcd; set < nsets; set += waves_per_xcd) {
        K key[kXcdChunks];
        uint64_t m[kXcdChunks];
#pragma unroll
        for (int k = 0; k < kXcdChunks; ++k) {
            const uint64_t qi = (set * kXcdChunks + k) * 64 + static_cast<uint64_t>(lane);
            const bool valid = qi < B;
            key[k] = valid ? q[qi] : K(0);
            uint32_t b = 0;
            if (nsplit) {
#pragma unroll
                for (int x = 0; x < kXcds - 1; ++x) b += split[x] < key[k] ? 1u : 0u;
            } else {
                b = static_cast<uint32_t>(qi % kXcds);
            }
            m[k] = __ballot(valid && b == xcd);
        }
        uint32_t left = 0;
#pragma unroll
        for (int k = 0; k < kXcdChunks; ++k) left += static_cast<uint32_t>(__popcll(m[k]));
        for (uint32_t r0 = 0; r0 < left; r0 += kGroups * QPG) {  // the same for the whole wave
            // group grp takes the selected queries of rank r0 + grp + 8 j
            K kk[QPG];
            uint64_t qq[QPG];
#pragma unroll
            for (int j = 0; j < QPG; ++j) {
                uint32_t rank = r0 + grp + kGroups * static_cast<uint32_t>(j);
                const bool live = rank < left;
                int chunk = 0, src = 0;
                if (live) {
#pragma unroll
                    for (int k = 0; k < kXcdChunks; ++k) {
                        const uint32_t c = static_cast<uint32_t>(__popcll(m[k]));
                        if (chunk == k && rank >= c) {
                            rank -= c;
                            chunk = k + 1;
                        }
                    }
                    src = nth_set_bit(m[chunk], rank);
                }
                // a cross-lane read returns the source lane's register, so
                // read every chunk's key there and keep the wanted one
                K kx = K(0);
#pragma unroll
                for (int k = 0; k < kXcdChunks; ++k) {
                    const K v = static_cast<K>(__shfl(key[k], src, 64));
                    if (chunk == k) kx = v;
                }
                kk[j] = kx;
                qq[j] = live ? (set * kXcdChunks + static_cast<uint64_t>(chunk)) * 64 + static_cast<uint64_t>(src)
                             : ~0ull;
            }
            uint32_t leaf[QPG];
            descend<K, G, QPG, false>(t, lds, mnodes, LV, kk, leaf, gl, gbase);
            finish_lookups<K, G, QPG, VC, NT>(t, kk, leaf, qq, empty, gl, gbase, vout, fout);
        }
    }
}

template <class K, int G, int LV>
__global__ __launch_bounds__(kLookupBlock) void k_range(TreeView<K> t, const K* __restrict__ lo,
                                                         const K* __restrict__ hi,
                                                         const uint32_t* __restrict__ maxc,
                                                         const uint64_t* __restrict__ off, uint64_t B,
                                                         K* __restrict__ okeys, K* __restrict__ ovals,
                                                         uint32_t* __restrict__ cnt_out, uint64_t ntiles) {
    using T = Trav<K, G>;
    constexpr int KPL = T::KPL;
    extern __shared__ __align__(16) uint8_t lds[];
    const uint8_t* mir = t.mirror;
    uint32_t mnodes = kMirrorMaxNodes;
    if constexpr (LV > 0) {
        mnodes = mirror_nodes_for_levels(LV);
        stage_mirror<K>(t.mirror, lds, mnodes);
        __syncthreads();
        mir = lds;
    }
    const MirrorHeader* mh = reinterpret_cast<const MirrorHeader*>(mir);
    const bool empty = mh->n_keys == 0;
    const int lane = lane_id();
    const int gl = lane % G, gbase = lane - gl;
    const uint64_t below_lanes = (1ull << gl) - 1ull;
    const uint64_t group = threadIdx.x / G;
    const uint64_t tile_q = kLookupBlock / G;
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint64_t qi = tile * tile_q + group;
        const bool live = qi < B;
        K key[1] = {live ? lo[qi] : K(0)};
        const K h = live ? hi[qi] : K(0);
        const uint32_t mx = live ? maxc[qi] : 0u;
        const uint64_t base = live ? off[qi] : 0ull;
        uint32_t leaf[1];
        descend<K, G, 1, false>(t, mir, mnodes, LV, key, leaf, gl, gbase);
        uint32_t c = 0;
        bool done = !live || empty || mx == 0 || key[0] > h;
        uint32_t cur = leaf[0];
        while (!done) {
            typename T::KV kv = T::load_keys(t.lkeys + static_cast<uint64_t>(cur) * kSlots, gl);
            typename T::KV vv = T::load_keys(t.lvals + static_cast<uint64_t>(cur) * kSlots, gl);
            const uint2 meta = t.lmeta[cur];
            bool ok[KPL];
            uint32_t within = 0, lanes_below = 0, total = 0;
            bool beyond = false;
            uint32_t pre[KPL];
#pragma unroll
            for (int e = 0; e < KPL; ++e) {
                const uint32_t slot = static_cast<uint32_t>(gl * KPL + e);
                const bool inl = slot < meta.x;
                ok[e] = inl && kv.v[e] >= key[0] && kv.v[e] <= h;
                const uint64_t bits = group_bits<G>(__ballot(ok[e]), gbase);
                const uint64_t over = group_bits<G>(__ballot(inl && kv.v[e] > h), gbase);
                beyond = beyond || over != 0;
                lanes_below += static_cast<uint32_t>(__popcll(bits & below_lanes));
                total += static_cast<uint32_t>(__popcll(bits));
                pre[e] = within;
                within += ok[e] ? 1u : 0u;
            }
#pragma unroll
            for (int e = 0; e < KPL; ++e) {
                if (ok[e]) {
                    const uint32_t p = c + lanes_below + pre[e];
                    if (p < mx) {
                        okeys[base + p] = kv.v[e];
                        ovals[base + p] = vv.v[e];
                    }
                }
            }
            c += total;
            done = c >= mx || beyond || meta.y == kNone || meta.x == 0;
            cur = meta.y;
        }
        if (live && gl == 0) cnt_out[qi] = c < mx ? c : mx;
    }
}

// ---------------------------------------------------------------- launch

static uint32_t lds_bytes_for(int lv, int key_bytes) {
    if (lv <= 0) return 0;
    uint32_t n = mirror_nodes_for_levels(lv);
    return key_bytes == 8 ? MirrorLayout<uint64_t>::bytes(n) : MirrorLayout<uint32_t>::bytes(n);
}

static uint64_t grid_for(uint64_t ntiles, int lv, int key_bytes) {
    // resident workgroups: 8 per CU when the mirror copy is small, fewer
    // when it takes a large share of the 160 KiB of LDS per CU
    uint32_t lds = lds_bytes_for(lv, key_bytes);
    uint64_t per_cu = 8;
    if (lds > 0) {
        uint64_t fit = (160u * 1024u) / lds;
        if (fit < per_cu) per_cu = fit < 1 ? 1 : fit;
    }
    uint64_t cap = 256 * per_cu;
    return ntiles < cap ? (ntiles < 1 ? 1 : ntiles) : cap;
}

template <class K, int G, int QPG, int LV, bool VC, int NT>
static void launch_lookup_t(const TreeView<K>& t, const K* q, uint64_t B, K* vout, uint8_t* fout, hipStream_t s) {
    const uint64_t tile_q = static_cast<uint64_t>(kLookupBlock / G) * QPG;
    const uint64_t ntiles = (B + tile_q - 1) / tile_q;
    const uint64_t grid = grid_for(ntiles, LV, sizeof(K));
    hipLaunchKernelGGL((k_lookup<K, G, QPG, LV, VC, NT>), dim3(static_cast<uint32_t>(grid)), dim3(kLookupBlock),
                       lds_bytes_for(LV, sizeof(K)), s, t, q, B, vout, fout, ntiles);
}

template <class K, bool VC, int NT>
static void launch_lookup_xcd(const TreeView<K>& t, const K* q, uint64_t B, K* vout, uint8_t* fout, hipStream_t s) {
    const uint64_t nchunks = (B + 63) / 64;
    // per XCD up to 256 workgroups (8 per CU) of four waves; every XCD reads
    // every chunk, four at a time per wave
    uint64_t per_xcd = (nchunks + 4 * kXcdChunks - 1) / (4 * kXcdChunks);
    if (per_xcd > 256) per_xcd = 256;
    if (per_xcd < 1) per_xcd = 1;
    hipLaunchKernelGGL((k_lookup_xcd<K, VC, NT>), dim3(static_cast<uint32_t>(per_xcd * kXcds)), dim3(kLookupBlock),
                       lds_bytes_for(2, sizeof(K)), s, t, q, B, vout, fout, nchunks);
}

template <class K, int G, int QPG, int LV>
static void launch_lookup_v(const TreeView<K>& t, const LaunchCfg& cfg, const K* q, uint64_t B, K* vout,
                            uint8_t* fout, hipStream_t s) {
    const bool xcd = cfg.xcd_split == 2 || (cfg.xcd_split == 1 && B >= kXcdMinBatch);
    // leaf lines read non-temporally: both (leaf_stream 1), none (2), or by
    // default the value line from kLargeBatch queries on
    const int nt = cfg.leaf_stream == 1 ? 3 : (cfg.leaf_stream == 0 && B >= kLargeBatch ? 2 : 0);
    if (xcd) {
        if (cfg.value_coload) {
            if (nt == 3) launch_lookup_xcd<K, true, 3>(t, q, B, vout, fout, s);
            else if (nt == 2) launch_lookup_xcd<K, true, 2>(t, q, B, vout, fout, s);
            else launch_lookup_xcd<K, true, 0>(t, q, B, vout, fout, s);
        } else {
            if (nt == 3) launch_lookup_xcd<K, false, 3>(t, q, B, vout, fout, s);
            else if (nt == 2) launch_lookup_xcd<K, false, 2>(t, q, B, vout, fout, s);
            else launch_lookup_xcd<K, false, 0>(t, q, B, vout, fout, s);
        }
        return;
    }
    if (cfg.value_coload) {
        if (nt == 3) launch_lookup_t<K, G, QPG, LV, true, 3>(t, q, B, vout, fout, s);
        else if (nt == 2) launch_lookup_t<K, G, QPG, LV, true, 2>(t, q, B, vout, fout, s);
        else launch_lookup_t<K, G, QPG, LV, true, 0>(t, q, B, vout, fout, s);
    } else {
        if (nt == 3) launch_lookup_t<K, G, QPG, LV, false, 3>(t, q, B, vout, fout, s);
        else if (nt == 2) launch_lookup_t<K, G, QPG, LV, false, 2>(t, q, B, vout, fout, s);
        else launch_lookup_t<K, G, QPG, LV, false, 0>(t, q, B, vout, fout, s);
    }
}

template <class K, int G, int QPG>
static void launch_lookup_lv(const TreeView<K>& t, const LaunchCfg& cfg, const K* q, uint64_t B, K* vout,
                             uint8_t* fout, hipStream_t s) {
    switch (cfg.lds_levels) {
        case 0: launch_lookup_v<K, G, QPG, 0>(t, cfg, q, B, vout, fout, s); break;
        case 1: launch_lookup_v<K, G, QPG, 1>(t, cfg, q, B, vout, fout, s); break;
        case 2: launch_lookup_v<K, G, QPG, 2>(t, cfg, q, B, vout, fout, s); break;
        default: launch_lookup_v<K, G, QPG, 3>(t, cfg, q, B, vout, fout, s); break;
    }
}

// Lookup shape by batch size, for the fields the caller did not fix
// (measured on 2^24 u64 keys): small batches are latency-bound and want
// 16 lanes per query, one query per group and no LDS staging (the top
// levels are L2 hits, the staging a barrier on the critical path); large
// batches are bound by the rate of L2 misses and want 8 lanes, two queries
// in flight per group (one is too few to hide the misses; four cost more in
// registers and barriers than they add) and the top two levels in LDS.
static LaunchCfg shape_for(const LaunchCfg& cfg, uint64_t B) {
    LaunchCfg c = cfg;
    int lanes, qpg, lds;
    if (B < kMidBatch) { lanes = 16; qpg = 1; lds = 0; }
    else if (B < kLargeBatch) { lanes = 8; qpg = 1; lds = 0; }
    else { lanes = 8; qpg = cfg.large_qpg ? cfg.large_qpg : 2; lds = 2; }
    if (cfg.shape_auto & 1) c.lanes = lanes;
    if (cfg.shape_auto & 2) c.queries_per_group = qpg;
    else if (B >= kLargeBatch && cfg.large_qpg) c.queries_per_group = cfg.large_qpg;
    if (cfg.shape_auto & 4) c.lds_levels = lds;
    return c;
}

template <class K>
void launch_lookup(const TreeView<K>& t, const LaunchCfg& cfg0, const K* q, uint64_t B, K* vout, uint8_t* fout,
                   hipStream_t s) {
    const LaunchCfg cfg = shape_for(cfg0, B);
    const int qpg = cfg.queries_per_group;
    switch (cfg.lanes) {
        case 4:
            if (qpg >= 4) launch_lookup_lv<K, 4, 4>(t, cfg, q, B, vout, fout, s);
            else if (qpg == 2) launch_lookup_lv<K, 4, 2>(t, cfg, q, B, vout, fout, s);
            else launch_lookup_lv<K, 4, 1>(t, cfg, q, B, vout, fout, s);
            break;
        case 16:
            if (qpg >= 4) launch_lookup_lv<K, 16, 4>(t, cfg, q, B, vout, fout, s);
            else if (qpg == 2) launch_lookup_lv<K, 16, 2>(t, cfg, q, B, vout, fout, s);
            else launch_lookup_lv<K, 16, 1>(t, cfg, q, B, vout, fout, s);
            break;
        default:
            if (qpg >= 4) launch_lookup_lv<K, 8, 4>(t, cfg, q, B, vout, fout, s);
            else if (qpg == 2) launch_lookup_lv<K, 8, 2>(t, cfg, q, B, vout, fout, s);
            else launch_lookup_lv<K, 8, 1>(t, cfg, q, B, vout, fout, s);
            break;
    }
}

template <class K, int G, int LV>
static void launch_range_t(const TreeView<K>& t, const K* lo, const K* hi, const uint32_t* mx, const uint64_t* off,
                           uint64_t B, K* ok, K* ov, uint32_t* cnt, hipStream_t s) {
    const uint64_t tile_q = kLookupBlock / G;
    const uint64_t ntiles = (B + tile_q - 1) / tile_q;
    const uint64_t grid = grid_for(ntiles, LV, sizeof(K));
    hipLaunchKernelGGL((k_range<K, G, LV>), dim3(static_cast<uint32_t>(grid)), dim3(kLookupBlock),
                       lds_bytes_for(LV, sizeof(K)), s, t, lo, hi, mx, off, B, ok, ov, cnt, ntiles);
}

template <class K, int G>
static void launch_range_lv(const TreeView<K>& t, int lv, const K* lo, const K* hi, const uint32_t* mx,
                            const uint64_t* off, uint64_t B, K* ok, K* ov, uint32_t* cnt, hipStream_t s) {
    switch (lv) {
        case 0: launch_range_t<K, G, 0>(t, lo, hi, mx, off, B, ok, ov, cnt, s); break;
        case 1: launch_range_t<K, G, 1>(t, lo, hi, mx, off, B, ok, ov, cnt, s); break;
        case 2: launch_range_t<K, G, 2>(t, lo, hi, mx, off, B, ok, ov, cnt, s); break;
        default: launch_range_t<K, G, 3>(t, lo, hi, mx, off, B, ok, ov, cnt, s); break;
    }
}

template <class K>
void launch_range(const TreeView<K>& t, const LaunchCfg& cfg, const K* lo, const K* hi, const uint32_t* mx,
                  const uint64_t* off, uint64_t B, K* ok, K* ov, uint32_t* cnt, hipStream_t s) {
    switch (cfg.lanes) {
        case 4: launch_range_lv<K, 4>(t, cfg.lds_levels, lo, hi, mx, off, B, ok, ov, cnt, s); break;
        case 16: launch_range_lv<K, 16>(t, cfg.lds_levels, lo, hi, mx, off, B, ok, ov, cnt, s); break;
        default: launch_range_lv<K, 8>(t, cfg.lds_levels, lo, hi, mx, off, B, ok, ov, cnt, s); break;
    }
}

template void launch_lookup<uint32_t>(const TreeView<uint32_t>&, const LaunchCfg&, const uint32_t*, uint64_t,
                                      uint32_t*, uint8_t*, hipStream_t);
template void launch_lookup<uint64_t>(const TreeView<uint64_t>&, const LaunchCfg&, const uint64_t*, uint64_t,
                                      uint64_t*, uint8_t*, hipStream_t);
template void launch_range<uint32_t>(const TreeView<uint32_t>&, const LaunchCfg&, const uint32_t*,
                                     const uint32_t*, const uint32_t*, const uint64_t*, uint64_t, uint32_t*,
                                     uint32_t*, uint32_t*, hipStream_t);
template void launch_range<uint64_t>(const TreeView<uint64_t>&, const LaunchCfg&, const uint64_t*,
                                     const uint64_t*, const uint32_t*, const uint64_t*, uint64_t, uint64_t*,
                                     uint64_t*, uint32_t*, hipStream_t);

}  // namespace gt
