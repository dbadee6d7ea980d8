// Static tree of the paper's key and node variants (layout in wide.h).
//
// Search (Sections IV-A, IV-E, IV-F): a query is served by a group of m
// lanes, one per node entry.  At an inner node lane s compares the query
// with entry s as a cascade over the key's 64-bit words taken most
// significant first (a word decides unless it is equal, as the paper's
// cascading priority comparison resolves its 32 per-byte comparators), and
// the group's ballot of "entry < query" counted by popcount is the priority
// encoder: the child is the first one whose entry is >= the query.  Inner
// entries are stored word-sliced, so a level first reads only the leading
// words and goes on to a further word only for entries that tie the query
// (and, for exact-match lookups, only where the node's tie mask says the
// tie does not decide).  The node's child range comes from one 16-byte
// record read in the same round as the leading words, so a level costs one
// dependent round unless an entry ties.  At the leaf each lane compares its
// key for equality; small batches read every entry's key and value in one
// round, large ones read the leading words first and only the lanes that
// tie read the rest of their entry and its value.  Large batches also give
// a query fewer lanes (8 or 16, each holding several entries), so that more
// queries are in flight per wave.  The first matching lane
// answers (the paper's 8-byte data), else the result is all ones with
// found = 0 (Section IV-D's -1).  Ranges descend with lo and walk the linked
// leaves (Section III).
//
// Build (Section V-B's one-time build, done on the device): the keys are
// sorted (8-byte keys by the library's radix sort; 32-byte keys by four
// stable radix sorts of one 64-bit word each, least significant word first,
// each pass reordering the permutation the previous ones produced), checked
// for duplicates, packed evenly into leaves of at most m - 1 keys, and the
// inner levels are packed bottom-up with at most m and (below the root) at
// least m/2 children (Section III).  At fill 1 and n = (m-1) * m^(h-1) keys
// that gives sum_{i<h} m^i nodes, Section III's N_max.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <algorithm>
#include <vector>

#include "common.h"
#include "prims.h"
#include "wide.h"

namespace gt {

namespace {

constexpr int kWBlock = 256;
constexpr uint32_t kWGridMax = 8192;
// batches from this size on are bound by the lines they read and by the
// queries in flight, not by the dependent rounds: fewer lanes per query and
// their leaves read in two rounds (k_wlookupg)
constexpr uint64_t kWTwoRound = 1u << 13;
// lanes per query of a large batch (k_wlookupg), by order: measured best at
// 2^20 queries, 8 lanes for orders 16 and 32, 16 for order 64
template <int M>
constexpr int large_lanes() { return M == 64 ? 16 : 8; }

// ---------------------------------------------------------------- keys

// A key as kw words ready to compare: an 8-byte key is its own integer; a
// 32-byte key's words are read big-endian, so that comparing the words in
// order compares the bytes in order.  `raw` keeps the bytes as stored.
template <int KW>
struct Key {
    uint64_t w[KW];
    uint64_t raw[KW];
};

template <int KW>
__device__ __forceinline__ Key<KW> load_key(const uint8_t* p) {
    Key<KW> k;
    if constexpr (KW == 1) {
        k.raw[0] = *reinterpret_cast<const uint64_t*>(p);
        k.w[0] = k.raw[0];
    } else {
        const uint4* q = reinterpret_cast<const uint4*>(p);
#pragma unroll
        for (int h = 0; h < KW / 2; ++h) {
            const uint4 a = q[h];
            k.raw[2 * h] = (static_cast<uint64_t>(a.y) << 32) | a.x;
            k.raw[2 * h + 1] = (static_cast<uint64_t>(a.w) << 32) | a.z;
        }
#pragma unroll
        for (int i = 0; i < KW; ++i) k.w[i] = __builtin_bswap64(k.raw[i]);
    }
    return k;
}

template <int KW>
__device__ __forceinline__ Key<KW> max_key() {
    Key<KW> k;
#pragma unroll
    for (int i = 0; i < KW; ++i) k.w[i] = k.raw[i] = ~0ull;
    return k;
}

// a < b: the first unequal word decides (cascade from the most significant)
template <int KW>
__device__ __forceinline__ bool key_less(const Key<KW>& a, const Key<KW>& b) {
    bool lt = a.w[KW - 1] < b.w[KW - 1];
#pragma unroll
    for (int i = KW - 2; i >= 0; --i) lt = (a.w[i] < b.w[i]) || (a.w[i] == b.w[i] && lt);
    return lt;
}

template <int KW>
__device__ __forceinline__ bool key_eq(const Key<KW>& a, const Key<KW>& b) {
    bool eq = true;
#pragma unroll
    for (int i = 0; i < KW; ++i) eq = eq && a.raw[i] == b.raw[i];
    return eq;
}

template <int KW>
__device__ __forceinline__ void store_key(uint8_t* p, const Key<KW>& k) {
    if constexpr (KW == 1) {
        *reinterpret_cast<uint64_t*>(p) = k.raw[0];
    } else {
        uint4* q = reinterpret_cast<uint4*>(p);
#pragma unroll
        for (int h = 0; h < KW / 2; ++h)
            q[h] = make_uint4(static_cast<uint32_t>(k.raw[2 * h]), static_cast<uint32_t>(k.raw[2 * h] >> 32),
                              static_cast<uint32_t>(k.raw[2 * h + 1]), static_cast<uint32_t>(k.raw[2 * h + 1] >> 32));
    }
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
    const uint32_t lo = shfl_u32(static_cast<uint32_t>(v), src);
    const uint32_t hi = shfl_u32(static_cast<uint32_t>(v >> 32), src);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// ------------------------------------------------------------- search

// Descend from the root to the leaf whose key range holds `key` (the first
// child whose entry is >= key at every level).  Every lane of the group
// takes part; `ref` ends as a leaf id.
// An inner node's entries are word-sliced: word w (0 = most significant,
// as a big-endian number) of its m entries sits in m consecutive 8-byte
// words, so a level reads the leading words alone (one 128-byte line at
// m = 16).  A lane whose leading word ties the query's goes on to the
// entry's other words (read together, one more round) -- the cascade of the
// paper's priority comparison, taken through memory -- unless the tie
// already decides: when the key after the entry in key order (the first of
// the next child) has a larger leading word, no key of a later child shares
// the query's leading word, so a present query lies at or below the entry.
// Exact-match lookups take that shortcut (bit s of the node's mask is set
// when it does not apply); range descents, which need the exact first key
// >= lo, compare in full.  Entries below the child count are sorted, so the
// "entry < query" lanes stay a prefix of the group either way.
template <int KW, int M, bool Exact>
__device__ __forceinline__ uint32_t descend(const WideView& v, const Key<KW>& key, bool valid, uint32_t root,
                                            uint32_t height, int s, int gbase) {
    const uint64_t* ik = reinterpret_cast<const uint64_t*>(v.ikeys);
    uint32_t ref = root;
    for (uint32_t d = 0; d + 1 < height; ++d) {
        const uint64_t base = static_cast<uint64_t>(ref) * KW * M + s;
        const uint64_t e0 = ik[base];
        const uint4 meta = v.imeta[ref];
        bool lt = e0 < key.w[0];
        if constexpr (KW > 1) {
            const uint64_t mask = Exact ? ~0ull : (static_cast<uint64_t>(meta.w) << 32 | meta.z);
            const bool need = valid && e0 == key.w[0] && ((mask >> s) & 1ull);
            if (__ballot(need)) {
                if (need) {
                    uint64_t e[KW];
#pragma unroll
                    for (int w = 1; w < KW; ++w) e[w] = ik[base + static_cast<uint64_t>(w) * M];
                    bool l = e[KW - 1] < key.w[KW - 1];
#pragma unroll
                    for (int w = KW - 2; w >= 1; --w) l = (e[w] < key.w[w]) || (e[w] == key.w[w] && l);
                    lt = l;
                }
            }
        }
        lt = valid && lt;
        const uint32_t ci = static_cast<uint32_t>(__popcll(group_bits<M>(__ballot(lt), gbase)));
        ref = meta.x + ci;
    }
    return ref;
}

// Leaves of 32-byte keys: per leaf, the m leading words (big-endian
// numbers), then m 32-byte records {words 1..3 as big-endian numbers,
// value}.  Leaves of 8-byte keys: lkeys[leaf][m] keys, lvals[leaf][m].
constexpr uint64_t kLeafEntry32 = 40;  // bytes per entry of a 32-byte-key leaf

template <int KW, int M>
__device__ __forceinline__ const uint64_t* leaf_words(const WideView& v, uint32_t leaf) {
    return reinterpret_cast<const uint64_t*>(v.lkeys + static_cast<uint64_t>(leaf) * M * (KW == 1 ? 8 : kLeafEntry32));
}

// words 1..3 and the value of entry s of a 32-byte-key leaf
template <int M>
__device__ __forceinline__ void leaf_record(const WideView& v, uint32_t leaf, int s, uint64_t (&w)[3], uint64_t& val) {
    const uint4* r = reinterpret_cast<const uint4*>(v.lkeys + static_cast<uint64_t>(leaf) * M * kLeafEntry32 + M * 8 +
                                                    static_cast<uint64_t>(s) * 32);
    const uint4 a = r[0], b = r[1];
    w[0] = (static_cast<uint64_t>(a.y) << 32) | a.x;
    w[1] = (static_cast<uint64_t>(a.w) << 32) | a.z;
    w[2] = (static_cast<uint64_t>(b.y) << 32) | b.x;
    val = (static_cast<uint64_t>(b.w) << 32) | b.z;
}

// entry s of a leaf as a key (and its value)
template <int KW, int M>
__device__ __forceinline__ Key<KW> leaf_entry(const WideView& v, uint32_t leaf, int s, uint64_t& val) {
    Key<KW> k;
    const uint64_t w0 = leaf_words<KW, M>(v, leaf)[s];
    if constexpr (KW == 1) {
        k.w[0] = k.raw[0] = w0;
        val = v.lvals[static_cast<uint64_t>(leaf) * M + s];
    } else {
        uint64_t w[3];
        leaf_record<M>(v, leaf, s, w, val);
        k.w[0] = w0;
#pragma unroll
        for (int i = 1; i < KW; ++i) k.w[i] = w[i - 1];
#pragma unroll
        for (int i = 0; i < KW; ++i) k.raw[i] = __builtin_bswap64(k.w[i]);
    }
    return k;
}

// Lookup of a small batch: M lanes per query, every entry of the leaf --
// key and value -- read in one round (large batches: k_wlookupg).
template <int KW, int M>
__global__ __launch_bounds__(kWBlock) void k_wlookup(WideView v, const uint8_t* __restrict__ q, uint64_t B,
                                                     uint64_t* __restrict__ vout, uint8_t* __restrict__ fout) {
    constexpr int QPW = 64 / M;
    constexpr uint64_t KB = 8 * KW;
    const int lane = threadIdx.x & 63, s = lane % M, gbase = lane - s;
    const uint64_t wave = (blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x) >> 6;
    const uint64_t nwaves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 6;
    const uint32_t root = v.hdr->root, height = v.hdr->height;
    const bool empty = v.hdr->n_keys == 0;
    for (uint64_t base = wave * QPW; base < B; base += nwaves * QPW) {
        const uint64_t i = base + lane / M;
        const bool valid = i < B;
        const Key<KW> key = valid ? load_key<KW>(q + i * KB) : max_key<KW>();
        const uint32_t leaf = descend<KW, M, false>(v, key, valid, root, height, s, gbase);
        // the padding repeats the last key, so the first equal slot is a
        // real one; an empty tree's one leaf holds only padding
        uint64_t val = 0;
        const Key<KW> lk = leaf_entry<KW, M>(v, leaf, s, val);
        const bool eq = valid && !empty && key_eq<KW>(lk, key);
        const uint64_t gb = group_bits<M>(__ballot(eq), gbase);
        const int f = gb ? __ffsll(static_cast<long long>(gb)) - 1 : 0;
        const uint64_t fv = shfl_u64(val, gbase + f);
        if (valid && s == 0) {
            vout[i] = gb ? fv : ~0ull;
            fout[i] = gb ? 1 : 0;
        }
    }
}

// Large batches: G lanes per query (64 / G queries per wave instead of
// 64 / M), lane l holding entries [l E, (l + 1) E) of a node, E = M / G.
// The leading words of a lane's entries are one vector load; the ballots of
// each entry position add up to the child index.
// Inner ties and the leaf follow k_wlookup's two-round rules: an inner
// entry whose leading word ties the query reads its other words only where
// the node's tie mask says the tie does not decide; at the leaf a lane
// reads the rest and the value of an entry whose leading word equals the
// query's; the first equal entry answers.
template <int KW, int M, int G>
__global__ __launch_bounds__(kWBlock) void k_wlookupg(WideView v, const uint8_t* __restrict__ q, uint64_t B,
                                                      uint64_t* __restrict__ vout, uint8_t* __restrict__ fout) {
    constexpr int E = M / G, QPW = 64 / G;
    constexpr uint64_t KB = 8 * KW;
    static_assert(E == 2 || E == 4 || E == 8, "two to eight entries per lane");
    const int lane = threadIdx.x & 63, gl = lane % G, gbase = lane - gl;
    const uint64_t wave = (blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x) >> 6;
    const uint64_t nwaves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 6;
    const uint32_t root = v.hdr->root, height = v.hdr->height;
    const bool empty = v.hdr->n_keys == 0;
    const uint64_t* ik = reinterpret_cast<const uint64_t*>(v.ikeys);
    for (uint64_t base = wave * QPW; base < B; base += nwaves * QPW) {
        const uint64_t i = base + lane / G;
        const bool valid = i < B;
        const Key<KW> key = valid ? load_key<KW>(q + i * KB) : max_key<KW>();
        uint32_t ref = root;
        for (uint32_t d = 0; d + 1 < height; ++d) {
            const uint64_t nb = static_cast<uint64_t>(ref) * KW * M + static_cast<uint64_t>(gl) * E;
            uint64_t e0[E];
            {
                const uint4* p4 = reinterpret_cast<const uint4*>(ik + nb);
#pragma unroll
                for (int h = 0; h < E / 2; ++h) {
                    const uint4 x = p4[h];
                    e0[2 * h] = (static_cast<uint64_t>(x.y) << 32) | x.x;
                    e0[2 * h + 1] = (static_cast<uint64_t>(x.w) << 32) | x.z;
                }
            }
            const uint4 meta = v.imeta[ref];
            uint32_t ci = 0;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                bool lt = e0[e] < key.w[0];
                if constexpr (KW > 1) {
                    const uint32_t slot = static_cast<uint32_t>(gl * E + e);
                    const uint64_t mask = (static_cast<uint64_t>(meta.w) << 32) | meta.z;
                    const bool need = valid && e0[e] == key.w[0] && ((mask >> slot) & 1ull);
                    if (need) {
                        uint64_t w[KW];
#pragma unroll
                        for (int x = 1; x < KW; ++x) w[x] = ik[nb + e + static_cast<uint64_t>(x) * M];
                        bool l = w[KW - 1] < key.w[KW - 1];
#pragma unroll
                        for (int x = KW - 2; x >= 1; --x) l = (w[x] < key.w[x]) || (w[x] == key.w[x] && l);
                        lt = l;
                    }
                }
                ci += static_cast<uint32_t>(__popcll(group_bits<G>(__ballot(valid && lt), gbase)));
            }
            ref = meta.x + ci;
        }
        // leaf: leading words of this lane's entries, then the rest and the
        // value of the entries that tie
        const uint64_t* lw = leaf_words<KW, M>(v, ref) + gl * E;
        uint64_t w0[E];
        {
            const uint4* p4 = reinterpret_cast<const uint4*>(lw);
#pragma unroll
            for (int h = 0; h < E / 2; ++h) {
                const uint4 x = p4[h];
                w0[2 * h] = (static_cast<uint64_t>(x.y) << 32) | x.x;
                w0[2 * h + 1] = (static_cast<uint64_t>(x.w) << 32) | x.z;
            }
        }
        int first = -1;
        uint64_t val = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            bool eq = valid && !empty && first < 0 && w0[e] == key.w[0];
            if (eq) {
                const int slot = gl * E + e;
                uint64_t vv;
                if constexpr (KW == 1) {
                    vv = v.lvals[static_cast<uint64_t>(ref) * M + slot];
                } else {
                    uint64_t w[3];
                    leaf_record<M>(v, ref, slot, w, vv);
#pragma unroll
                    for (int x = 1; x < KW; ++x) eq = eq && w[x - 1] == key.w[x];
                }
                if (eq) {
                    first = e;
                    val = vv;
                }
            }
        }
        // the padding repeats the last key, so the first equal entry is a
        // real one: the lowest lane with a match holds it
        const uint64_t gb = group_bits<G>(__ballot(first >= 0), gbase);
        const int f = gb ? __ffsll(static_cast<long long>(gb)) - 1 : 0;
        const uint64_t fv = shfl_u64(val, gbase + f);
        if (valid && gl == 0) {
            vout[i] = gb ? fv : ~0ull;
            fout[i] = gb ? 1 : 0;
        }
    }
}

template <int KW, int M>
__global__ __launch_bounds__(kWBlock) void k_wrange(WideView v, const uint8_t* __restrict__ lo,
                                                    const uint8_t* __restrict__ hi, const uint32_t* __restrict__ maxc,
                                                    const uint64_t* __restrict__ off, uint64_t B,
                                                    uint8_t* __restrict__ okeys, uint64_t* __restrict__ ovals,
                                                    uint32_t* __restrict__ cnt) {
    constexpr int QPW = 64 / M;
    constexpr uint64_t KB = 8 * KW;
    const int lane = threadIdx.x & 63, s = lane % M, gbase = lane - s;
    const uint64_t wave = (blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x) >> 6;
    const uint64_t nwaves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 6;
    const uint32_t root = v.hdr->root, height = v.hdr->height;
    const bool empty = v.hdr->n_keys == 0;
    for (uint64_t base = wave * QPW; base < B; base += nwaves * QPW) {
        const uint64_t i = base + lane / M;
        const bool valid = i < B;
        const Key<KW> a = valid ? load_key<KW>(lo + i * KB) : max_key<KW>();
        const Key<KW> b = valid ? load_key<KW>(hi + i * KB) : max_key<KW>();
        const uint32_t mx = valid ? maxc[i] : 0u;
        const uint64_t o = valid ? off[i] : 0ull;
        uint32_t leaf = descend<KW, M, true>(v, a, valid, root, height, s, gbase);
        uint32_t c = 0;
        bool active = valid && !empty && mx > 0 && !key_less<KW>(b, a);
        // walk the chain; the loop runs while any group of the wave is active
        while (__ballot(active)) {
            bool stop = true;
            if (active) {
                const uint2 meta = v.lmeta[leaf];
                uint64_t val;
                const Key<KW> k = leaf_entry<KW, M>(v, leaf, s, val);
                const bool real = static_cast<uint32_t>(s) < meta.x;
                const bool above = real && key_less<KW>(b, k);
                const bool in = real && !key_less<KW>(k, a) && !above;
                const uint64_t ib = group_bits<M>(__ballot(in), gbase);
                const uint64_t ab = group_bits<M>(__ballot(above), gbase);
                const uint32_t rank = static_cast<uint32_t>(__popcll(ib & ((1ull << s) - 1ull)));
                if (in && c + rank < mx) {
                    store_key<KW>(okeys + (o + c + rank) * KB, k);
                    ovals[o + c + rank] = val;
                }
                c += static_cast<uint32_t>(__popcll(ib));
                stop = ab != 0 || c >= mx || meta.y == kNone;
                leaf = meta.y;
            }
            // every quantity above is the same on all lanes of a group, so
            // a group stops as a whole
            active = active && !stop;
        }
        if (valid && s == 0) cnt[i] = c < mx ? c : mx;
    }
}

// -------------------------------------------------------------- build

// word w (0 = most significant) of 32-byte key perm[i], read big-endian
__global__ void k_word_of(const uint8_t* __restrict__ keys, const uint32_t* __restrict__ perm, int w, uint64_t n,
                          uint64_t* __restrict__ out) {
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint64_t src = perm ? perm[i] : i;
        out[i] = __builtin_bswap64(*reinterpret_cast<const uint64_t*>(keys + src * 32 + w * 8));
    }
}

// out[i] = perm[idx[i]] (perm null: the identity)
__global__ void k_compose(const uint32_t* __restrict__ perm, const uint32_t* __restrict__ idx, uint64_t n,
                          uint32_t* __restrict__ out) {
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        out[i] = perm ? perm[idx[i]] : idx[i];
}

// the pairs in sorted order; flag |= 1 when two neighbours are equal
template <int KW>
__global__ void k_wgather(const uint8_t* __restrict__ keys, const uint64_t* __restrict__ vals,
                          const uint32_t* __restrict__ perm, uint64_t n, uint8_t* __restrict__ sk,
                          uint64_t* __restrict__ sv) {
    constexpr uint64_t KB = 8 * KW;
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint64_t src = perm[i];
        store_key<KW>(sk + i * KB, load_key<KW>(keys + src * KB));
        sv[i] = vals[src];
    }
}

template <int KW>
__global__ void k_wdup(const uint8_t* __restrict__ sk, uint64_t n, uint32_t* flag) {
    constexpr uint64_t KB = 8 * KW;
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i + 1 < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        if (key_eq<KW>(load_key<KW>(sk + i * KB), load_key<KW>(sk + (i + 1) * KB))) atomicOr(flag, 1u);
}

// leaf j holds sorted pairs [j n / L, (j+1) n / L); its largest key goes to
// maxk[j]
template <int KW, int M>
__global__ void k_wleaves(uint8_t* __restrict__ lkeys, uint64_t* __restrict__ lvals, uint2* __restrict__ lmeta,
                          const uint8_t* __restrict__ sk, const uint64_t* __restrict__ sv, uint64_t n, uint64_t L,
                          uint8_t* __restrict__ maxk, uint64_t* __restrict__ succ) {
    constexpr uint64_t KB = 8 * KW;
    for (uint64_t t = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; t < L * M;
         t += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint64_t j = t / M, s = t % M;
        const uint64_t b = part_start(j, n, L), e = part_start(j + 1, n, L), c = e - b;
        Key<KW> k = c ? load_key<KW>(sk + (b + (s < c ? s : c - 1)) * KB) : max_key<KW>();
        const uint64_t val = s < c ? sv[b + s] : ~0ull;
        if constexpr (KW == 1) {
            store_key<KW>(lkeys + t * KB, k);
            lvals[t] = val;
        } else {
            uint8_t* lb = lkeys + j * M * kLeafEntry32;
            reinterpret_cast<uint64_t*>(lb)[s] = k.w[0];
            uint4* r = reinterpret_cast<uint4*>(lb + M * 8 + s * 32);
            r[0] = make_uint4(static_cast<uint32_t>(k.w[1]), static_cast<uint32_t>(k.w[1] >> 32),
                              static_cast<uint32_t>(k.w[2]), static_cast<uint32_t>(k.w[2] >> 32));
            r[1] = make_uint4(static_cast<uint32_t>(k.w[3]), static_cast<uint32_t>(k.w[3] >> 32),
                              static_cast<uint32_t>(val), static_cast<uint32_t>(val >> 32));
        }
        if (s == 0) {
            lmeta[j] = make_uint2(static_cast<uint32_t>(c), j + 1 < L ? static_cast<uint32_t>(j + 1) : kNone);
            store_key<KW>(maxk + j * KB, c ? load_key<KW>(sk + (e - 1) * KB) : max_key<KW>());
            // leading word of the key after the leaf's last one (all ones
            // past the end)
            succ[j] = e < n ? load_key<KW>(sk + e * KB).w[0] : ~0ull;
        }
    }
}

// P nodes over the C nodes of the level below (ids child_base + ...):
// node j holds children [j C / P, (j+1) C / P); entry s < c-1 is child s's
// largest key, later entries the largest key value
template <int KW, int M>
__global__ void k_winner(uint8_t* __restrict__ ikeys, uint4* __restrict__ imeta,
                         const uint8_t* __restrict__ cmax, const uint64_t* __restrict__ csucc, uint64_t C, uint64_t P,
                         uint32_t node_base, uint8_t* __restrict__ nmax, uint64_t* __restrict__ nsucc) {
    constexpr uint64_t KB = 8 * KW;
    // the stride is a multiple of 64 and M divides 64, so a node's M
    // entries are M consecutive lanes of one wave in every pass
    const int lane = threadIdx.x & 63, gbase = lane - lane % M;
    for (uint64_t t = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; t < P * M;
         t += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint64_t j = t / M, s = t % M;
        const uint64_t b = part_start(j, C, P), e = part_start(j + 1, C, P), c = e - b;
        const Key<KW> k = (s + 1 < c) ? load_key<KW>(cmax + (b + s) * KB) : max_key<KW>();
        // word-sliced: word w of entry s at ((node * KW) + w) * M + s, as a
        // big-endian number (the order the search compares in)
        uint64_t* ik = reinterpret_cast<uint64_t*>(ikeys);
#pragma unroll
        for (int w = 0; w < KW; ++w) ik[((node_base + j) * KW + w) * M + s] = k.w[w];
        // the entry's leading word is shared with the next key in key order
        const bool shared = s + 1 < c && k.w[0] == csucc[b + s];
        const uint64_t bits = group_bits<M>(__ballot(shared), gbase);
        if (s == 0) {
            imeta[node_base + j] = make_uint4(static_cast<uint32_t>(b), static_cast<uint32_t>(c),
                                              static_cast<uint32_t>(bits), static_cast<uint32_t>(bits >> 32));
            store_key<KW>(nmax + j * KB, load_key<KW>(cmax + (e - 1) * KB));
            nsucc[j] = csucc[e - 1];
        }
    }
}

__global__ void k_wheader(WideHeader* h, uint32_t height, uint64_t n, uint32_t ni, uint32_t nl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        h->root = 0;
        h->height = height;
        h->n_keys = n;
        h->n_inner = ni;
        h->n_leaves = nl;
        h->error = 0;
    }
}

uint32_t grid_for(uint64_t items, int block) {
    const uint64_t g = (items + block - 1) / block;
    return static_cast<uint32_t>(std::max<uint64_t>(1, std::min<uint64_t>(g, 65536)));
}

// ------------------------------------------------------------ host side

constexpr uint64_t kAl = 256;
uint64_t al(uint64_t x) { return (x + kAl - 1) / kAl * kAl; }

int orders_ok(int kb, int m) {
    if (kb == 32) return m == 16 || m == 32 || m == 64;
    if (kb == 8) return m == 32 || m == 64;
    return 0;
}

int order_of(const gt_params* p) { return p->fanout ? static_cast<int>(p->fanout) : 16; }
double fill_of_w(const gt_params* p) { return p->fill == 0.0f ? 1.0 : static_cast<double>(p->fill); }

// nodes a level of `items` entries packs into: at most cap * fill per node,
// at least ceil(cap / 2) each when there are two or more
uint64_t wpack(uint64_t items, uint64_t cap, double fill) {
    uint64_t per = static_cast<uint64_t>(static_cast<double>(cap) * fill);
    if (per < 1) per = 1;
    const uint64_t a = (items + per - 1) / per, b = items / ((cap + 1) / 2);
    const uint64_t c = a < b ? a : b;
    return c < 1 ? 1 : c;
}

// level sizes, leaves first
std::vector<uint64_t> wlevels(uint64_t n, int m, double fill) {
    std::vector<uint64_t> v{wpack(n, static_cast<uint64_t>(m - 1), fill)};
    while (v.back() > 1) v.push_back(wpack(v.back(), static_cast<uint64_t>(m), fill));
    return v;
}

struct WSizes {
    uint64_t leaves, inner, bytes;
    int height;
};

WSizes wsizes(int kb, int m, uint64_t n, double fill) {
    const std::vector<uint64_t> lv = wlevels(n, m, fill);
    WSizes z{};
    z.leaves = lv[0];
    for (size_t i = 1; i < lv.size(); ++i) z.inner += lv[i];
    z.height = static_cast<int>(lv.size());
    const uint64_t ni = z.inner ? z.inner : 1;
    // leaves: 8-byte keys and values in two arrays, or 40 bytes per entry
    // of a 32-byte-key leaf in one
    const uint64_t lk = kb == 32 ? z.leaves * m * kLeafEntry32 : z.leaves * m * 8;
    const uint64_t lvb = kb == 32 ? 0 : z.leaves * m * 8;
    z.bytes = al(sizeof(WideHeader)) + al(ni * m * kb) + al(ni * 16) + al(lk) + al(lvb) + al(z.leaves * 8);
    return z;
}

template <int KW, int M>
void launch_wlookup(const WideView& v, const void* keys, uint64_t B, void* vout, uint8_t* fout, hipStream_t s) {
    constexpr uint64_t qpb = kWBlock / M;
    const uint64_t g = std::min<uint64_t>((B + qpb - 1) / qpb, kWGridMax);
    if (B >= kWTwoRound) {
        constexpr int G = large_lanes<M>();
        constexpr uint64_t qpbg = kWBlock / G;
        const uint64_t gg = std::min<uint64_t>((B + qpbg - 1) / qpbg, kWGridMax);
        hipLaunchKernelGGL((k_wlookupg<KW, M, G>), dim3(static_cast<uint32_t>(gg)), dim3(kWBlock), 0, s, v,
                           reinterpret_cast<const uint8_t*>(keys), B, reinterpret_cast<uint64_t*>(vout), fout);
    } else {
        hipLaunchKernelGGL((k_wlookup<KW, M>), dim3(static_cast<uint32_t>(g)), dim3(kWBlock), 0, s, v,
                           reinterpret_cast<const uint8_t*>(keys), B, reinterpret_cast<uint64_t*>(vout), fout);
    }
}

template <int KW, int M>
void launch_wrange(const WideView& v, const void* lo, const void* hi, const uint32_t* maxc, const uint64_t* off,
                   uint64_t B, void* ok, void* ov, uint32_t* cnt, hipStream_t s) {
    constexpr uint64_t qpb = kWBlock / M;
    const uint64_t g = std::min<uint64_t>((B + qpb - 1) / qpb, kWGridMax);
    hipLaunchKernelGGL((k_wrange<KW, M>), dim3(static_cast<uint32_t>(g)), dim3(kWBlock), 0, s, v,
                       reinterpret_cast<const uint8_t*>(lo), reinterpret_cast<const uint8_t*>(hi), maxc, off, B,
                       reinterpret_cast<uint8_t*>(ok), reinterpret_cast<uint64_t*>(ov), cnt);
}

template <int KW, int M>
void launch_wpack(WideTree* w, const uint8_t* sk, const uint64_t* sv, uint64_t n, const std::vector<uint64_t>& lv,
                  uint8_t* maxa, uint8_t* maxb, uint64_t* succa, uint64_t* succb, hipStream_t s) {
    const uint64_t L = lv[0];
    hipLaunchKernelGGL((k_wleaves<KW, M>), dim3(grid_for(L * M, kWBlock)), dim3(kWBlock), 0, s, w->lkeys, w->lvals,
                       w->lmeta, sk, sv, n, L, maxa, succa);
    // inner ids top-down: the level just above the leaves gets the last ids
    uint64_t below = L;
    uint64_t base = w->inner_cap;
    uint8_t* cur = maxa;
    uint8_t* nxt = maxb;
    uint64_t* scur = succa;
    uint64_t* snxt = succb;
    for (size_t l = 1; l < lv.size(); ++l) {
        const uint64_t P = lv[l];
        base -= P;
        hipLaunchKernelGGL((k_winner<KW, M>), dim3(grid_for(P * M, kWBlock)), dim3(kWBlock), 0, s, w->ikeys, w->imeta,
                           cur, scur, below, P, static_cast<uint32_t>(base), nxt, snxt);
        std::swap(cur, nxt);
        std::swap(scur, snxt);
        below = P;
    }
}

// child ids in imeta are relative to the level below; make them absolute
// inner ids for inner children (leaf children keep their leaf ids)
void fix_child_bases(WideTree* w, const std::vector<uint64_t>& lv, hipStream_t s);

__global__ void k_rebase(uint4* imeta, uint32_t first, uint32_t count, uint32_t add) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        imeta[first + i].x += add;
}

void fix_child_bases(WideTree* w, const std::vector<uint64_t>& lv, hipStream_t s) {
    // level l (l >= 2) occupies ids [base_l, base_l + lv[l]); its children
    // are the level below, ids starting at base_{l-1}
    std::vector<uint64_t> base(lv.size(), 0);
    uint64_t b = w->inner_cap;
    for (size_t l = 1; l < lv.size(); ++l) {
        b -= lv[l];
        base[l] = b;
    }
    for (size_t l = 2; l < lv.size(); ++l)
        hipLaunchKernelGGL(k_rebase, dim3(grid_for(lv[l], kWBlock)), dim3(kWBlock), 0, s, w->imeta,
                           static_cast<uint32_t>(base[l]), static_cast<uint32_t>(lv[l]),
                           static_cast<uint32_t>(base[l - 1]));
}

#define WHIP(x)                                    \
    do {                                           \
        if ((x) != hipSuccess) return GT_ERR_HIP;  \
    } while (0)

WideView view_of(const WideTree* w) {
    WideView v;
    v.hdr = w->hdr;
    v.ikeys = w->ikeys;
    v.imeta = w->imeta;
    v.lkeys = w->lkeys;
    v.lvals = w->lvals;
    v.lmeta = w->lmeta;
    return v;
}

// 32-byte keys are read and written with 16-byte accesses
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

template <class F>
bool dispatch(int kw, int m, F&& f) {
    if (kw == 1 && m == 32) { f(std::integral_constant<int, 1>{}, std::integral_constant<int, 32>{}); return true; }
    if (kw == 1 && m == 64) { f(std::integral_constant<int, 1>{}, std::integral_constant<int, 64>{}); return true; }
    if (kw == 4 && m == 16) { f(std::integral_constant<int, 4>{}, std::integral_constant<int, 16>{}); return true; }
    if (kw == 4 && m == 32) { f(std::integral_constant<int, 4>{}, std::integral_constant<int, 32>{}); return true; }
    if (kw == 4 && m == 64) { f(std::integral_constant<int, 4>{}, std::integral_constant<int, 64>{}); return true; }
    return false;
}

}  // namespace

bool wide_selected(const gt_params* p) {
    return p && (p->key_bytes == 32 || (p->key_bytes == 8 && (p->fanout == 32 || p->fanout == 64)));
}

bool wide_params_ok(const gt_params* p) {
    if (!wide_selected(p)) return false;
    const int m = order_of(p);
    if (!orders_ok(static_cast<int>(p->key_bytes), m)) return false;
    if (p->leaf_cap != 0 && p->leaf_cap != static_cast<uint32_t>(m - 1)) return false;
    if (p->fill != 0.0f && (p->fill < 0.5f || p->fill > 1.0f)) return false;
    // the search shape is fixed by the order; these apply to the fanout-16 tree only
    if (p->lanes_per_query || p->lds_levels || p->sorted_mode || p->queries_per_group || p->value_coload ||
        p->xcd_split || p->leaf_stream || p->reserved)
        return false;
    return true;
}

uint64_t wide_arena_bytes(const gt_params* p, uint64_t n) {
    if (!wide_params_ok(p)) return 0;
    return wsizes(static_cast<int>(p->key_bytes), order_of(p), n, fill_of_w(p)).bytes;
}

gt_status wide_build(const gt_params* p, const void* keys, const void* values, uint64_t n, void* arena,
                     uint64_t arena_bytes, hipStream_t s, WideTree** out) {
    if (!wide_params_ok(p) || !arena || !out || (n && (!keys || !values))) return GT_ERR_INVALID;
    if (n >= (1ull << 31)) return GT_ERR_INVALID;
    if (p->key_bytes == 32 && n && !aligned16(keys)) return GT_ERR_INVALID;
    if (!aligned16(arena)) return GT_ERR_INVALID;
    const int kb = static_cast<int>(p->key_bytes), kw = kb / 8, m = order_of(p);
    const double fill = fill_of_w(p);
    const WSizes z = wsizes(kb, m, n, fill);
    if (z.bytes > arena_bytes) return GT_ERR_CAPACITY;
    if (z.height > kMaxLevels) return GT_ERR_CAPACITY;
    const std::vector<uint64_t> lv = wlevels(n, m, fill);

    WideTree* w = new WideTree();
    w->kw = kw;
    w->m = m;
    w->fill = fill;
    w->inner_cap = z.inner;
    w->leaf_cap = z.leaves;
    w->height = static_cast<uint32_t>(z.height);
    uint8_t* a = reinterpret_cast<uint8_t*>(arena);
    uint64_t o = 0;
    const uint64_t ni = z.inner ? z.inner : 1;
    w->hdr = reinterpret_cast<WideHeader*>(a + o); o += al(sizeof(WideHeader));
    w->ikeys = a + o; o += al(ni * m * kb);
    w->imeta = reinterpret_cast<uint4*>(a + o); o += al(ni * 16);
    if (kw == 4) {
        w->lkeys = a + o; o += al(z.leaves * m * kLeafEntry32);
        w->lvals = nullptr;
    } else {
        w->lkeys = a + o; o += al(z.leaves * m * 8);
        w->lvals = reinterpret_cast<uint64_t*>(a + o); o += al(z.leaves * m * 8);
    }
    w->lmeta = reinterpret_cast<uint2*>(a + o); o += al(z.leaves * 8);
    w->arena_bytes = o;

    // temporary buffers: sorted keys and values, the permutation and its
    // ping-pong, one word column (the sort's input) with the sort's output
    // and ping-pong, sort scratch, level maxima (two levels), the duplicate /
    // sort-failure flag
    const uint64_t nn = n ? n : 1;
    const uint64_t b_keys = al(nn * kb), b_vals = al(nn * 8), b_idx = al(nn * 4), b_word = al(nn * 8);
    const uint64_t b_sort = al(sort_tmp_bytes(nn, 8)), b_max = al(z.leaves * kb), b_succ = al(z.leaves * 8);
    const uint64_t total = b_keys + b_vals + 4 * b_idx + 3 * b_word + b_sort + 2 * b_max + 2 * b_succ + kAl;
    uint8_t* tmp = nullptr;
    if (hipMalloc(&tmp, total) != hipSuccess) {
        delete w;
        return GT_ERR_HIP;
    }
    uint8_t* q = tmp;
    uint8_t* sk = q; q += b_keys;
    uint64_t* sv = reinterpret_cast<uint64_t*>(q); q += b_vals;
    uint32_t* perm = reinterpret_cast<uint32_t*>(q); q += b_idx;
    uint32_t* perm2 = reinterpret_cast<uint32_t*>(q); q += b_idx;
    uint32_t* si = reinterpret_cast<uint32_t*>(q); q += b_idx;
    uint32_t* si2 = reinterpret_cast<uint32_t*>(q); q += b_idx;
    uint64_t* col = reinterpret_cast<uint64_t*>(q); q += b_word;
    uint64_t* col2 = reinterpret_cast<uint64_t*>(q); q += b_word;
    uint64_t* colsrc = reinterpret_cast<uint64_t*>(q); q += b_word;
    void* stmp = q; q += b_sort;
    uint8_t* maxa = q; q += b_max;
    uint8_t* maxb = q; q += b_max;
    uint64_t* succa = reinterpret_cast<uint64_t*>(q); q += b_succ;
    uint64_t* succb = reinterpret_cast<uint64_t*>(q); q += b_succ;
    uint32_t* flag = reinterpret_cast<uint32_t*>(q);

    gt_status st = GT_OK;
    uint32_t hflag = 0;
    do {
        if (hipMemsetAsync(flag, 0, 4, s) != hipSuccess) { st = GT_ERR_HIP; break; }
        if (n) {
            const uint8_t* kin = reinterpret_cast<const uint8_t*>(keys);
            if (kw == 1) {
                // one radix sort of the integers; positions come from the sort
                sort_from<uint64_t>(reinterpret_cast<const uint64_t*>(kin), col, perm, col2, si2, n, stmp, s, flag,
                                    2u);
            } else {
                // least significant word first; each stable pass reorders the
                // permutation the previous passes left
                uint32_t* cur = nullptr;
                for (int wd = kw - 1; wd >= 0; --wd) {
                    hipLaunchKernelGGL(k_word_of, dim3(grid_for(n, kWBlock)), dim3(kWBlock), 0, s, kin, cur, wd, n,
                                       colsrc);
                    sort_from<uint64_t>(colsrc, col, si, col2, si2, n, stmp, s, flag, 2u);
                    uint32_t* dst = (cur == perm) ? perm2 : perm;
                    hipLaunchKernelGGL(k_compose, dim3(grid_for(n, kWBlock)), dim3(kWBlock), 0, s, cur, si, n, dst);
                    cur = dst;
                }
                if (cur != perm)
                    if (hipMemcpyAsync(perm, cur, n * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) {
                        st = GT_ERR_HIP;
                        break;
                    }
            }
            const bool four = kw == 4;
            if (four) {
                hipLaunchKernelGGL((k_wgather<4>), dim3(grid_for(n, kWBlock)), dim3(kWBlock), 0, s, kin,
                                   reinterpret_cast<const uint64_t*>(values), perm, n, sk, sv);
                hipLaunchKernelGGL((k_wdup<4>), dim3(grid_for(n, kWBlock)), dim3(kWBlock), 0, s, sk, n, flag);
            } else {
                hipLaunchKernelGGL((k_wgather<1>), dim3(grid_for(n, kWBlock)), dim3(kWBlock), 0, s, kin,
                                   reinterpret_cast<const uint64_t*>(values), perm, n, sk, sv);
                hipLaunchKernelGGL((k_wdup<1>), dim3(grid_for(n, kWBlock)), dim3(kWBlock), 0, s, sk, n, flag);
            }
        }
        if (hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            st = GT_ERR_HIP;
            break;
        }
        if (hflag & 2u) { st = GT_ERR_DEVICE; break; }  // a sort gave up its bounded wait
        if (hflag) { st = GT_ERR_DUPLICATE; break; }
        dispatch(kw, m, [&](auto KWc, auto Mc) {
            launch_wpack<decltype(KWc)::value, decltype(Mc)::value>(w, sk, sv, n, lv, maxa, maxb, succa, succb, s);
        });
        fix_child_bases(w, lv, s);
        hipLaunchKernelGGL(k_wheader, dim3(1), dim3(64), 0, s, w->hdr, static_cast<uint32_t>(z.height), n,
                           static_cast<uint32_t>(z.inner), static_cast<uint32_t>(z.leaves));
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) st = GT_ERR_HIP;
    } while (0);
    (void)hipStreamSynchronize(s);
    (void)hipFree(tmp);
    if (st != GT_OK) {
        delete w;
        return st;
    }
    *out = w;
    return GT_OK;
}

gt_status wide_lookup(const WideTree* w, const void* keys, uint64_t B, void* values_out, uint8_t* found_out,
                      hipStream_t s) {
    if (w->kw == 4 && !aligned16(keys)) return GT_ERR_INVALID;
    const WideView v = view_of(w);
    dispatch(w->kw, w->m, [&](auto KWc, auto Mc) {
        launch_wlookup<decltype(KWc)::value, decltype(Mc)::value>(v, keys, B, values_out, found_out, s);
    });
    return hipGetLastError() == hipSuccess ? GT_OK : GT_ERR_HIP;
}

gt_status wide_range(const WideTree* w, const void* lo, const void* hi, const uint32_t* max_out,
                     const uint64_t* out_offsets, uint64_t B, void* out_keys, void* out_values, uint32_t* count_out,
                     hipStream_t s) {
    if (w->kw == 4 && (!aligned16(lo) || !aligned16(hi) || !aligned16(out_keys))) return GT_ERR_INVALID;
    const WideView v = view_of(w);
    dispatch(w->kw, w->m, [&](auto KWc, auto Mc) {
        launch_wrange<decltype(KWc)::value, decltype(Mc)::value>(v, lo, hi, max_out, out_offsets, B, out_keys,
                                                                 out_values, count_out, s);
    });
    return hipGetLastError() == hipSuccess ? GT_OK : GT_ERR_HIP;
}

gt_status wide_stats(const WideTree* w, gt_tree_stats* out, hipStream_t s) {
    WideHeader h;
    WHIP(hipMemcpyAsync(&h, w->hdr, sizeof h, hipMemcpyDeviceToHost, s));
    WHIP(hipStreamSynchronize(s));
    memset(out, 0, sizeof *out);
    out->n_keys = h.n_keys;
    out->height = h.height;
    out->root = h.height > 1 ? 0u : kLeafTag;
    out->inner_used = h.n_inner;
    out->inner_cap = w->inner_cap;
    out->leaf_used = h.n_leaves;
    out->leaf_cap = w->leaf_cap;
    out->arena_bytes = w->arena_bytes;
    out->max_batch = 0;
    out->error_word = h.error;
    out->key_bytes = static_cast<uint32_t>(8 * w->kw);
    return GT_OK;
}

gt_status wide_device_error(const WideTree* w, hipStream_t s) {
    uint32_t e = 0;
    WHIP(hipMemcpyAsync(&e, &w->hdr->error, 4, hipMemcpyDeviceToHost, s));
    WHIP(hipStreamSynchronize(s));
    return e ? GT_ERR_DEVICE : GT_OK;
}

gt_status wide_export(const WideTree* w, void* host_buf, uint64_t* bytes, hipStream_t s) {
    WideHeader h;
    WHIP(hipMemcpyAsync(&h, w->hdr, sizeof h, hipMemcpyDeviceToHost, s));
    WHIP(hipStreamSynchronize(s));
    const uint64_t kb = 8 * static_cast<uint64_t>(w->kw), m = static_cast<uint64_t>(w->m), C = m - 1;
    const uint64_t ni = h.n_inner, nl = h.n_leaves;
    const uint64_t rin = m * (kb + 4), rlf = C * (kb + 8) + 8;
    const uint64_t need = 48 + ni * rin + nl * rlf;
    if (!host_buf) {
        *bytes = need;
        return GT_OK;
    }
    if (*bytes < need) return GT_ERR_CAPACITY;
    const uint64_t lkb = w->kw == 4 ? nl * m * kLeafEntry32 : nl * m * kb;
    std::vector<uint8_t> ik(ni * m * kb), lk(lkb);
    std::vector<uint4> im(ni);
    std::vector<uint2> lm(nl);
    std::vector<uint64_t> lvv(nl * m);
    if (ni) {
        WHIP(hipMemcpyAsync(ik.data(), w->ikeys, ik.size(), hipMemcpyDeviceToHost, s));
        WHIP(hipMemcpyAsync(im.data(), w->imeta, ni * 16, hipMemcpyDeviceToHost, s));
    }
    if (nl) {
        WHIP(hipMemcpyAsync(lk.data(), w->lkeys, lk.size(), hipMemcpyDeviceToHost, s));
        if (w->kw == 1) WHIP(hipMemcpyAsync(lvv.data(), w->lvals, nl * m * 8, hipMemcpyDeviceToHost, s));
        WHIP(hipMemcpyAsync(lm.data(), w->lmeta, nl * 8, hipMemcpyDeviceToHost, s));
    }
    WHIP(hipStreamSynchronize(s));
    // inner levels top-down; the nodes whose children are leaves are the
    // last level of ids: those with ids past every inner child reference
    // (the level just above the leaves holds the largest ids)
    std::vector<uint64_t> lv = wlevels(h.n_keys, w->m, w->fill);
    const uint64_t leaf_parents_first = ni - (lv.size() > 1 ? lv[1] : 0);
    uint8_t* o = reinterpret_cast<uint8_t*>(host_buf);
    const uint32_t root = h.height > 1 ? 0u : kLeafTag;
    const uint32_t hdr[10] = {0x58455447u, static_cast<uint32_t>(kb), static_cast<uint32_t>(m),
                              static_cast<uint32_t>(C), h.height, root, nl ? 0u : kNone,
                              static_cast<uint32_t>(ni), static_cast<uint32_t>(nl), 8u};
    memcpy(o, hdr, 40);
    memcpy(o + 40, &h.n_keys, 8);
    o += 48;
    const uint64_t kw = static_cast<uint64_t>(w->kw);
    for (uint64_t i = 0; i < ni; ++i) {
        // inner entries back from word slices to key bytes: a 32-byte key's
        // words are big-endian numbers, an 8-byte key's word is native
        for (uint64_t j = 0; j < m; ++j)
            for (uint64_t wd = 0; wd < kw; ++wd) {
                uint64_t x;
                memcpy(&x, ik.data() + ((i * kw + wd) * m + j) * 8, 8);
                if (kw > 1) x = __builtin_bswap64(x);
                memcpy(o + j * kb + wd * 8, &x, 8);
            }
        uint32_t* ch = reinterpret_cast<uint32_t*>(o + m * kb);
        const bool leaf_kids = i >= leaf_parents_first;
        for (uint64_t j = 0; j < m; ++j) {
            uint32_t r = kNone;
            if (j < im[i].y) r = (leaf_kids ? kLeafTag : 0u) | (im[i].x + static_cast<uint32_t>(j));
            memcpy(ch + j, &r, 4);
        }
        o += rin;
    }
    for (uint64_t i = 0; i < nl; ++i) {
        if (w->kw == 1) {
            memcpy(o, lk.data() + i * m * kb, C * kb);
            memcpy(o + C * kb, lvv.data() + i * m, C * 8);
        } else {
            // leading word and record back to key bytes (big-endian words)
            const uint8_t* lb = lk.data() + i * m * kLeafEntry32;
            for (uint64_t j = 0; j < C; ++j) {
                uint64_t x[5];
                memcpy(&x[0], lb + j * 8, 8);
                memcpy(&x[1], lb + m * 8 + j * 32, 32);
                for (int wd = 0; wd < 4; ++wd) {
                    const uint64_t be = __builtin_bswap64(x[wd]);
                    memcpy(o + j * kb + wd * 8, &be, 8);
                }
                memcpy(o + C * kb + j * 8, &x[4], 8);
            }
        }
        memcpy(o + C * (kb + 8), &lm[i], 8);
        o += rlf;
    }
    *bytes = need;
    return GT_OK;
}

}  // namespace gt
