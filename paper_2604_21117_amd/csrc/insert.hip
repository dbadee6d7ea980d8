// Insert batches: sort, deduplicate, locate, plan, check, apply.  Delete
// batches (the last section of this file) share the sort, deduplication
// and locate, then remove keys in place and merge what fell below half full.
//
// The paper searches a static tree (Section V-A); inserts are the dynamic
// counterpart that keeps Section III's invariants: sorted leaves, equal
// leaf depth, every non-root node at least half full.  The batch behaves
// like inserting its pairs one at a time in batch order: a present key is
// overwritten, and the last occurrence of a key in the batch supplies its
// value.
//
//  1. Sort (key, batch index) stably; run heads are the distinct keys; the
//     last element of each run holds the final value.  Every non-head is
//     UPDATED.
//  2. Locate: each distinct key descends the tree (the lookup traversal of
//     traverse.h) recording the inner node and child slot per level; a key
//     found in its leaf is an update, the others are new.
//  3. Plan, read-only, level by level from the leaves up.  Touched leaves
//     are the runs of new keys with the same leaf; a leaf with c old and r
//     new keys gets t = c + r entries and splits into ceil(t/16) pieces when
//     t > 16 (even sizes, so every piece holds >= 8).  Touched parents are
//     the runs of touched children with the same parent; a parent whose
//     children split gains sum(k-1) entries and splits the same way.  Piece
//     counts are scanned into allocation offsets, so new node ids follow key
//     order and repeated runs give the same tree.
//  4. Check: if the node pools cannot hold every new node the device error
//     word gets the capacity bit and nothing below runs (the batch is
//     applied whole or not at all).
//  5. Apply: updates in place; one wave per touched leaf merges its old keys
//     (held in registers) with its new keys and writes the pieces, the first
//     in place, the others to new leaves linked into the chain; then one wave
//     per changed parent, level by level, rebuilds its entry list (old
//     entries shifted, split children replaced by their pieces and piece
//     separators) and writes its own pieces.  A root that splits grows new
//     levels above it, packed with the same even rule.
//  6. Commit the header (key count, pool cursors, height, root) and refresh
//     the top-levels mirror.
#include <atomic>

#include "insert.h"
#include "lanes.h"
#include "mirror.h"
#include "prims.h"
#include "traverse.h"

namespace gt {

constexpr int kBlk = 256;

struct InsState {
    uint32_t U, R;
    uint32_t ok;
    uint32_t height;       // tree height when the batch started
    uint32_t overflow;     // item pool would overflow (internal error)
    uint32_t grow_nodes, grow_levels, new_root;
    uint32_t mirror_dirty;
    uint32_t lvl_count[kMaxLevels];  // items per level (0 = leaves)
    uint32_t lvl_base[kMaxLevels];   // first item of the level in the pool
    uint32_t lvl_new[kMaxLevels];    // new nodes the level's items create
    uint32_t lvl_alloc[kMaxLevels];  // first new id of the level
    uint32_t lvl_psep[kMaxLevels];   // first piece separator of the level
    uint32_t deleted;      // delete batch: keys removed
    uint32_t rebuild;      // delete batch: a parent would fall below half full
    uint32_t merges;       // delete batch: leaf runs left below half full (listed in f1)
    uint32_t gmerges;      // delete batch: parents that would fall below half full (listed in upos)
    uint32_t pad[3];
};

template <class K>
struct Ins {
    InsState* st;
    K* sk; K* sk2; uint32_t* si; uint32_t* si2; void* sort_tmp;
    uint32_t* f0; uint32_t* f1; void* scan_tmp;
    K* uk; K* uv; uint32_t* upos; uint32_t* uleaf; uint8_t* uslot; uint8_t* ufound;
    uint32_t* pn; uint8_t* pi; uint8_t* pc;  // per level: node, child slot taken, node's children
    uint8_t* ulc;                             // per distinct key: its leaf's key count
    K* nk; K* nv; uint32_t* nleaf; uint32_t* nu;
    uint32_t* it_node; uint32_t* it_rep; uint32_t* it_first; uint32_t* it_end;
    uint32_t* it_cold; uint32_t* it_k; uint32_t* it_off;
    uint8_t* it_cs;  // slot of the item's node in its parent
    K* psep;
    K* gsep0; K* gsep1; uint32_t* gid0; uint32_t* gid1;
    uint64_t Bm, ip_cap, ps_cap;
};

// ------------------------------------------------------------ scratch sizing

static uint64_t al(uint64_t x) { return (x + 255) / 256 * 256; }

static uint64_t item_pool_cap(uint64_t Bm, uint64_t leaf_cap) {
    uint64_t total = 0, lv = leaf_cap;
    for (int d = 0; d < kMaxLevels; ++d) {
        uint64_t bound = lv + 2;
        total += bound < Bm ? bound : Bm;
        lv = lv / 8;
    }
    return total;
}

static uint64_t psep_cap(uint64_t leaf_cap, uint64_t inner_cap) { return leaf_cap + inner_cap + 64; }

// items level d can hold (the item pool's per-level bound)
static uint64_t level_items_bound(uint64_t Bm, uint64_t leaf_cap, int d) {
    uint64_t lv = leaf_cap;
    for (int i = 0; i < d; ++i) lv /= 8;
    return lv + 2 < Bm ? lv + 2 : Bm;
}

template <class K>
static uint64_t carve(Ins<K>* v, uint8_t* base, uint64_t Bm, uint64_t leaf_cap, uint64_t inner_cap) {
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        uint8_t* p = base ? base + off : nullptr;
        off += al(bytes);
        return p;
    };
    const uint64_t ip = item_pool_cap(Bm, leaf_cap), ps = psep_cap(leaf_cap, inner_cap);
    Ins<K> x;
    x.Bm = Bm; x.ip_cap = ip; x.ps_cap = ps;
    x.st = reinterpret_cast<InsState*>(take(sizeof(InsState)));
    x.sk = reinterpret_cast<K*>(take(Bm * sizeof(K)));
    x.sk2 = reinterpret_cast<K*>(take(Bm * sizeof(K)));
    x.si = reinterpret_cast<uint32_t*>(take(Bm * 4));
    x.si2 = reinterpret_cast<uint32_t*>(take(Bm * 4));
    x.sort_tmp = take(sort_tmp_bytes(Bm, sizeof(K)));
    x.f0 = reinterpret_cast<uint32_t*>(take((Bm + 1) * 4));
    x.f1 = reinterpret_cast<uint32_t*>(take((Bm + 1) * 4));
    x.scan_tmp = take(scan_tmp_bytes(Bm + 1));
    x.uk = reinterpret_cast<K*>(take(Bm * sizeof(K)));
    x.uv = reinterpret_cast<K*>(take(Bm * sizeof(K)));
    x.upos = reinterpret_cast<uint32_t*>(take(Bm * 4));
    x.uleaf = reinterpret_cast<uint32_t*>(take(Bm * 4));
    x.uslot = take(Bm);
    x.ufound = take(Bm);
    x.pn = reinterpret_cast<uint32_t*>(take(static_cast<uint64_t>(kMaxLevels) * Bm * 4));
    x.pi = take(static_cast<uint64_t>(kMaxLevels) * Bm);
    x.pc = take(static_cast<uint64_t>(kMaxLevels) * Bm);
    x.ulc = take(Bm);
    x.nk = reinterpret_cast<K*>(take(Bm * sizeof(K)));
    x.nv = reinterpret_cast<K*>(take(Bm * sizeof(K)));
    x.nleaf = reinterpret_cast<uint32_t*>(take(Bm * 4));
    x.nu = reinterpret_cast<uint32_t*>(take(Bm * 4));
    x.it_node = reinterpret_cast<uint32_t*>(take(ip * 4));
    x.it_rep = reinterpret_cast<uint32_t*>(take(ip * 4));
    x.it_first = reinterpret_cast<uint32_t*>(take(ip * 4));
    x.it_end = reinterpret_cast<uint32_t*>(take(ip * 4));
    x.it_cold = reinterpret_cast<uint32_t*>(take(ip * 4));
    x.it_k = reinterpret_cast<uint32_t*>(take(ip * 4));
    x.it_off = reinterpret_cast<uint32_t*>(take(ip * 4));
    x.it_cs = take(ip);
    x.psep = reinterpret_cast<K*>(take(ps * sizeof(K)));
    x.gsep0 = reinterpret_cast<K*>(take(ps * sizeof(K)));
    x.gsep1 = reinterpret_cast<K*>(take(ps * sizeof(K)));
    x.gid0 = reinterpret_cast<uint32_t*>(take(ps * 4));
    x.gid1 = reinterpret_cast<uint32_t*>(take(ps * 4));
    if (v) *v = x;
    return off;
}

uint64_t insert_scratch_bytes(uint64_t max_batch, int key_bytes, uint64_t leaf_cap, uint64_t inner_cap) {
    if (key_bytes == 8) return carve<uint64_t>(nullptr, nullptr, max_batch, leaf_cap, inner_cap);
    return carve<uint32_t>(nullptr, nullptr, max_batch, leaf_cap, inner_cap);
}

// ------------------------------------------------------------------ kernels

__device__ __forceinline__ uint64_t gtid() { return blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; }
__device__ __forceinline__ uint64_t gstride() { return static_cast<uint64_t>(gridDim.x) * blockDim.x; }

// Clear the batch state (one workgroup).
template <class K>
__global__ void k_init(Ins<K> v, const DevHeader* hdr) {
    uint32_t* s = reinterpret_cast<uint32_t*>(v.st);
    for (uint32_t i = threadIdx.x; i < sizeof(InsState) / 4; i += blockDim.x) s[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) v.st->height = hdr->height;
}

template <class K>
__global__ void k_heads(Ins<K> v, uint64_t B, uint8_t* __restrict__ status) {
    for (uint64_t p = gtid(); p < B; p += gstride()) {
        const bool head = p == 0 || v.sk[p] != v.sk[p - 1];
        v.f0[p] = head ? 1u : 0u;
        if (!head) status[v.si[p]] = 1;  // UPDATED: an earlier occurrence exists
    }
}

template <class K>
__global__ void k_unique(Ins<K> v, uint64_t B, const K* __restrict__ vals) {
    for (uint64_t p = gtid(); p < B; p += gstride()) {
        const uint32_t f = v.f0[p], e = v.f1[p];
        if (f) {
            v.uk[e] = v.sk[p];
            v.upos[e] = static_cast<uint32_t>(p);
        }
        const bool last = p + 1 == B || v.sk[p + 1] != v.sk[p];
        if (last) v.uv[e + f - 1] = vals[v.si[p]];  // the run's last writer
    }
}

// Locate every distinct key; G lanes per key, QPG keys in flight per group,
// the top levels from LDS; NT threads per workgroup.
template <class K, int G, int QPG, int LV, int NT>
__device__ __forceinline__ void ph_locate(TreeView<K> t, Ins<K> v, uint8_t* __restrict__ status) {
    using T = Trav<K, G>;
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
    const uint64_t U = v.st->U;
    const int lane = lane_id();
    const int gl = lane % G, gbase = lane - gl;
    const uint64_t group = threadIdx.x / G;
    const uint64_t per_block = static_cast<uint64_t>(NT / G) * QPG;
    const uint64_t ntiles = (U + per_block - 1) / per_block;
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        K key[QPG];
        uint64_t qi[QPG];
#pragma unroll
        for (int j = 0; j < QPG; ++j) {
            const uint64_t u = tile * per_block + group * QPG + j;
            key[j] = u < U ? v.uk[u] : K(0);
            qi[j] = u < U ? u : ~0ull;
        }
        uint32_t leaf[QPG];
        descend<K, G, QPG, true>(t, mir, mnodes, LV, key, leaf, gl, gbase, v.pn, v.pi, v.Bm, qi, v.pc);
        typename T::KV kv[QPG];
        uint32_t lcnt[QPG];
#pragma unroll
        for (int j = 0; j < QPG; ++j) {
            kv[j] = T::load_keys(t.lkeys + static_cast<uint64_t>(leaf[j]) * kSlots, gl);
            lcnt[j] = t.lmeta[leaf[j]].x;
        }
#pragma unroll
        for (int j = 0; j < QPG; ++j) {
            const uint32_t slot = T::match_slot(kv[j], key[j], gbase);
            const bool found = slot < kSlots && !empty;
            if (qi[j] != ~0ull && gl == 0) {
                const uint64_t u = qi[j];
                v.ufound[u] = found ? 1 : 0;
                v.uleaf[u] = leaf[j];
                v.ulc[u] = static_cast<uint8_t>(lcnt[j]);
                v.uslot[u] = static_cast<uint8_t>(found ? slot : 0);
                v.f0[u] = found ? 0u : 1u;
                status[v.si[v.upos[u]]] = found ? 1 : 0;
            }
        }
    }
}

template <class K, int G, int QPG, int LV>
__global__ __launch_bounds__(kBlk) void k_locate(TreeView<K> t, Ins<K> v, uint8_t* __restrict__ status) {
    ph_locate<K, G, QPG, LV, kBlk>(t, v, status);
}

template <class K>
__device__ __forceinline__ void ph_compact_new(Ins<K> v, uint64_t tid, uint64_t nth) {
    const uint64_t U = v.st->U;
    for (uint64_t u = tid; u < U; u += nth) {
        if (!v.ufound[u]) {
            const uint32_t r = v.f1[u];
            v.nk[r] = v.uk[u];
            v.nv[r] = v.uv[u];
            v.nleaf[r] = v.uleaf[u];
            v.nu[r] = static_cast<uint32_t>(u);
        }
    }
}

template <class K>
__global__ void k_compact_new(Ins<K> v) {
    ph_compact_new<K>(v, gtid(), gstride());
}

template <class K>
__device__ __forceinline__ void ph_leaf_heads(Ins<K> v, uint64_t tid, uint64_t nth) {
    const uint64_t R = v.st->R;
    for (uint64_t r = tid; r < R; r += nth)
        v.f0[r] = (r == 0 || v.nleaf[r] != v.nleaf[r - 1]) ? 1u : 0u;
}

template <class K>
__global__ void k_leaf_heads(Ins<K> v) {
    ph_leaf_heads<K>(v, gtid(), gstride());
}

template <class K>
__device__ __forceinline__ void ph_leaf_items(Ins<K> v, uint64_t tid, uint64_t nth) {
    const uint64_t R = v.st->R;
    for (uint64_t r = tid; r < R; r += nth) {
        const uint32_t f = v.f0[r], e = v.f1[r];
        if (f) {
            if (e >= v.ip_cap) { v.st->overflow = 1; continue; }
            v.it_node[e] = v.nleaf[r];
            v.it_rep[e] = v.nu[r];
            v.it_first[e] = static_cast<uint32_t>(r);
        }
        if (r + 1 == R || v.f0[r + 1]) {
            const uint32_t seg = e + f - 1;
            if (seg < v.ip_cap) v.it_end[seg] = static_cast<uint32_t>(r + 1);
        }
    }
}

template <class K>
__global__ void k_leaf_items(Ins<K> v) {
    ph_leaf_items<K>(v, gtid(), gstride());
}

template <class K>
__device__ __forceinline__ void ph_leaf_plan(TreeView<K> t, Ins<K> v, uint64_t tid, uint64_t nth) {
    const uint64_t T0 = v.st->lvl_count[0];
    const int h = static_cast<int>(v.st->height);
    for (uint64_t i = tid; i < T0; i += nth) {
        if (h >= 2) v.it_cs[i] = v.pi[static_cast<uint64_t>(h - 2) * v.Bm + v.it_rep[i]];
        const uint32_t c = t.lmeta[v.it_node[i]].x;
        const uint64_t total = static_cast<uint64_t>(c) + (v.it_end[i] - v.it_first[i]);
        const uint32_t k = split_pieces(total);
        v.it_cold[i] = c;
        v.it_k[i] = k;
        v.f0[i] = k - 1;
    }
}

template <class K>
__global__ void k_leaf_plan(TreeView<K> t, Ins<K> v) {
    ph_leaf_plan<K>(t, v, gtid(), gstride());
}

// heads of the level-d items: runs of level-(d-1) items with the same parent
template <class K>
__device__ __forceinline__ void ph_par_heads(Ins<K> v, int d, uint64_t tid, uint64_t nth) {
    const int h = static_cast<int>(v.st->height);
    const int l = h - 1 - d;  // parent level, 0 = root level
    const uint64_t n = v.st->lvl_count[d - 1];
    const uint32_t b = v.st->lvl_base[d - 1];
    if (tid == 0) {
        v.st->lvl_base[d] = b + v.st->lvl_count[d - 1];
        v.st->lvl_psep[d] = v.st->lvl_psep[d - 1] + v.st->lvl_new[d - 1];
    }
    for (uint64_t i = tid; i < n; i += nth) {
        uint32_t f = 0;
        if (l >= 0) {
            const uint32_t p = v.pn[static_cast<uint64_t>(l) * v.Bm + v.it_rep[b + i]];
            f = (i == 0 || p != v.pn[static_cast<uint64_t>(l) * v.Bm + v.it_rep[b + i - 1]]) ? 1u : 0u;
        }
        v.f0[i] = f;
    }
}

template <class K>
__global__ void k_par_heads(Ins<K> v, int d) {
    ph_par_heads<K>(v, d, gtid(), gstride());
}

template <class K>
__device__ __forceinline__ void ph_par_items(Ins<K> v, int d, uint64_t tid, uint64_t nth) {
    const int h = static_cast<int>(v.st->height);
    const int l = h - 1 - d;
    if (l < 0) return;
    const uint64_t n = v.st->lvl_count[d - 1];
    const uint32_t b = v.st->lvl_base[d - 1];
    const uint32_t bd = v.st->lvl_base[d];
    for (uint64_t i = tid; i < n; i += nth) {
        const uint32_t f = v.f0[i], e = v.f1[i];
        if (f) {
            if (bd + e >= v.ip_cap) { v.st->overflow = 1; continue; }
            v.it_node[bd + e] = v.pn[static_cast<uint64_t>(l) * v.Bm + v.it_rep[b + i]];
            v.it_rep[bd + e] = v.it_rep[b + i];
            v.it_first[bd + e] = static_cast<uint32_t>(i);
        }
        if (i + 1 == n || v.f0[i + 1]) {
            const uint32_t seg = e + f - 1;
            if (bd + seg < v.ip_cap) v.it_end[bd + seg] = static_cast<uint32_t>(i + 1);
        }
    }
}

template <class K>
__global__ void k_par_items(Ins<K> v, int d) {
    ph_par_items<K>(v, d, gtid(), gstride());
}

template <class K>
__device__ __forceinline__ void ph_par_plan(TreeView<K> t, Ins<K> v, int d, uint64_t tid, uint64_t nth) {
    const uint64_t n = v.st->lvl_count[d];
    const uint32_t bd = v.st->lvl_base[d];
    const uint32_t bc = v.st->lvl_base[d - 1];
    const int lp = static_cast<int>(v.st->height) - 2 - d;  // tree level of the items' parents
    for (uint64_t j = tid; j < n; j += nth) {
        if (lp >= 0) v.it_cs[bd + j] = v.pi[static_cast<uint64_t>(lp) * v.Bm + v.it_rep[bd + j]];
        const uint32_t node = v.it_node[bd + j];
        uint32_t C = 0;
        const uint32_t* ch = t.ichild + static_cast<uint64_t>(node) * kSlots;
        for (int s = 0; s < kSlots; ++s) C += ch[s] != kNone ? 1u : 0u;
        uint64_t a = 0;
        for (uint32_t i = v.it_first[bd + j]; i < v.it_end[bd + j]; ++i) a += v.it_k[bc + i] - 1;
        const uint32_t k = split_pieces(C + a);
        v.it_cold[bd + j] = C;
        v.it_k[bd + j] = k;
        v.f0[j] = k - 1;
    }
}

template <class K>
__global__ void k_par_plan(TreeView<K> t, Ins<K> v, int d) {
    ph_par_plan<K>(t, v, d, gtid(), gstride());
}

// this level's allocation offsets, moved to the level's slice of the pool
template <class K>
__device__ __forceinline__ void ph_par_off(Ins<K> v, int d, uint64_t tid, uint64_t nth) {
    const uint64_t n = v.st->lvl_count[d];
    const uint32_t bd = v.st->lvl_base[d];
    for (uint64_t j = tid; j < n; j += nth) v.it_off[bd + j] = v.f1[j];
}

template <class K>
__global__ void k_par_off(Ins<K> v, int d) {
    ph_par_off<K>(v, d, gtid(), gstride());
}

// Capacity check and allocation bases (one thread).
template <class K>
__device__ __forceinline__ void ph_check(TreeView<K> t, Ins<K> v, uint64_t tid, uint64_t nth) {
    if (tid != 0) return;
    InsState* st = v.st;
    DevHeader* hdr = t.hdr;
    const int h = static_cast<int>(st->height);
    // root growth: the root is the level-(h-1) item, if touched
    uint32_t gn = 0, gl = 0;
    const int dr = h - 1;
    if (st->lvl_count[dr] > 0) {
        uint64_t cnt = v.it_k[st->lvl_base[dr]];
        while (cnt > 1) {
            const uint64_t nodes = cnt <= kSlots ? 1 : (cnt + kSlots - 1) / kSlots;
            gn += static_cast<uint32_t>(nodes);
            gl += 1;
            cnt = nodes;
        }
    }
    const uint64_t leaf_new = st->lvl_new[0];
    uint64_t inner_new = gn, sep_total = 0;
    for (int d = 0; d < h; ++d) sep_total += st->lvl_new[d];
    for (int d = 1; d < h; ++d) inner_new += st->lvl_new[d];
    bool ok = !st->overflow;
    if (hdr->error & kErrInternal) ok = false;  // e.g. the batch's device sort gave up
    if (hdr->leaf_used + leaf_new > t.leaf_cap) ok = false;
    if (hdr->inner_used + inner_new > t.inner_cap) ok = false;
    if (sep_total + 1 > v.ps_cap) ok = false;
    if (h + gl > kMaxLevels) ok = false;
    if (!ok && !(hdr->error & kErrInternal)) atomicOr(&hdr->error, st->overflow ? kErrInternal : kErrCapacity);
    st->ok = ok ? 1u : 0u;
    st->grow_nodes = gn;
    st->grow_levels = gl;
    st->lvl_alloc[0] = hdr->leaf_used;
    uint32_t cur = hdr->inner_used;
    for (int d = 1; d < h; ++d) {
        st->lvl_alloc[d] = cur;
        cur += st->lvl_new[d];
    }
    st->new_root = cur;  // first growth node id
}

template <class K>
__global__ void k_check(TreeView<K> t, Ins<K> v) {
    ph_check<K>(t, v, gtid(), gstride());
}

template <class K>
__global__ void k_apply_updates(TreeView<K> t, Ins<K> v) {
    if (!v.st->ok) return;
    const uint64_t U = v.st->U;
    for (uint64_t u = gtid(); u < U; u += gstride())
        if (v.ufound[u]) t.lvals[static_cast<uint64_t>(v.uleaf[u]) * kSlots + v.uslot[u]] = v.uv[u];
}

// first index in a[0..n) whose key is >= k
template <class K>
__device__ __forceinline__ uint32_t lower_bound_dev(const K* a, uint32_t n, K k) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < k) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// part_start and part_of for the splits the rebuilds make: below 2^16
// entries every product j * total fits in 32 bits, and a 32-bit division is
// a few instructions where a 64-bit one is a long sequence (a rebuild makes
// several per entry).  Same results; larger counts take the 64-bit forms.
__device__ __forceinline__ uint32_t pstart(uint64_t j, uint64_t total, uint64_t parts) {
    if (total < (1u << 16)) {
        return static_cast<uint32_t>(j) * static_cast<uint32_t>(total) / static_cast<uint32_t>(parts);
    }
    return static_cast<uint32_t>(part_start(j, total, parts));
}

__device__ __forceinline__ uint32_t ppart(uint64_t pos, uint64_t total, uint64_t parts) {
    if (total < (1u << 16)) {
        const uint32_t p = static_cast<uint32_t>(pos), t = static_cast<uint32_t>(total),
                       n = static_cast<uint32_t>(parts);
        uint32_t j = p * n / t;
        while (j + 1 < n && (j + 1) * t / n <= p) ++j;
        while (j > 0 && j * t / n > p) --j;
        return j;
    }
    return static_cast<uint32_t>(part_of(pos, total, parts));
}

// Lanes that rebuild one node (a leaf or an inner node): one per slot, four
// nodes per wave, so a wave keeps four nodes' reads in flight.
constexpr int kNodeLanes = 16;
static_assert(kNodeLanes == 16, "a node's lane group is one DPP row (row_lane)");

// Merge-split of the touched leaves: kNodeLanes lanes per leaf, group grp
// of ngrp.
// The planned items a rebuild reads: the arrays in device memory, or a copy
// in LDS that the one-workgroup apply makes of every level's items at its
// start (the plan wrote them all before; a rebuild only reads them), so
// that a level's rebuild waits on one round of device memory fewer.
struct ItemView {
    const uint32_t* node;
    const uint32_t* first;
    const uint32_t* end;
    const uint32_t* cold;
    const uint32_t* k;
    const uint32_t* off;
    const uint8_t* cs;
};

template <class K>
__device__ __forceinline__ ItemView items_in(const Ins<K>& v) {
    return ItemView{v.it_node, v.it_first, v.it_end, v.it_cold, v.it_k, v.it_off, v.it_cs};
}

template <class K>
__device__ __forceinline__ void apply_leaves_body(TreeView<K> t, Ins<K> v, uint64_t grp, uint64_t ngrp,
                                                  const ItemView& iv) {
    const uint32_t ok = v.st->ok;
    const uint64_t T0 = v.st->lvl_count[0];
    if (!ok || T0 == 0) return;
    const int gl = lane_id() % kNodeLanes, gbase = lane_id() - gl;
    const uint32_t alloc = v.st->lvl_alloc[0];
    for (uint64_t it = grp; it < T0; it += ngrp) {
        const uint32_t leaf = iv.node[it];
        const uint32_t first = iv.first[it];
        const uint32_t r = iv.end[it] - first;
        const uint32_t c = iv.cold[it];
        const uint32_t k = iv.k[it];
        const uint32_t off = iv.off[it];
        const uint32_t total = c + r;  // r is at most the batch size
        const uint32_t base_new = alloc + off;
        const K okey = t.lkeys[static_cast<uint64_t>(leaf) * kSlots + gl];
        const K oval = t.lvals[static_cast<uint64_t>(leaf) * kSlots + gl];
        const uint2 meta = t.lmeta[leaf];
        __threadfence_block();  // the old leaf is in registers before any write
        const K* nk = v.nk + first;
        const K* nv = v.nv + first;
        // one run of new keys (the common case): each lane holds at most one
        // old and one new element, and the group pads the pieces together
        const bool one_run = r <= static_cast<uint32_t>(kNodeLanes);
        auto place = [&](uint32_t pos, K key, K val) {
            const uint32_t j = ppart(pos, total, k);
            const uint32_t s0 = pstart(j, total, k), s1 = pstart(j + 1, total, k);
            const uint32_t slot = pos - s0;
            const uint64_t dest = j == 0 ? leaf : base_new + j - 1;
            t.lkeys[dest * kSlots + slot] = key;
            t.lvals[dest * kSlots + slot] = val;
            if (pos + 1 == s1) {
                const uint32_t cnt = static_cast<uint32_t>(s1 - s0);
                if (!one_run) {
                    for (uint32_t s = cnt; s < kSlots; ++s) {
                        t.lkeys[dest * kSlots + s] = key;
                        t.lvals[dest * kSlots + s] = kmax<K>();
                    }
                }
                const uint32_t nxt = (j + 1 < k) ? static_cast<uint32_t>(base_new + j) : meta.y;
                t.lmeta[dest] = make_uint2(cnt, nxt);
                if (j + 1 < k) v.psep[off + j] = key;
            }
        };
        const bool has_old = gl < static_cast<int>(c);
        uint64_t opos = ~0ull;
        if (one_run) {
            // new keys below this lane's old key, from the group's lanes
            // (a group is a row of 16 lanes: the moves are row broadcasts)
            const K mine = static_cast<uint32_t>(gl) < r ? nk[gl] : K(0);
            uint32_t below = 0;
            static_for<0, kNodeLanes>([&](auto S) {
                const K ks = row_lane<decltype(S)::value>(mine);
                below += (static_cast<uint32_t>(decltype(S)::value) < r && ks < okey) ? 1u : 0u;
            });
            if (has_old) opos = gl + below;
        } else if (has_old) {
            opos = gl + lower_bound_dev(nk, r, okey);
        }
        if (has_old) place(opos, okey, oval);
        uint64_t npos = ~0ull;
        K nkey = K(0);
        for (uint32_t q0 = 0; q0 < r; q0 += kNodeLanes) {
            const uint32_t q = q0 + gl;
            const bool act = q < r;
            const K key = act ? nk[q] : K(0);
            uint32_t rank = 0;
            static_for<0, kNodeLanes>([&](auto S) {
                const K ks = row_lane<decltype(S)::value>(okey);
                rank += (static_cast<uint32_t>(decltype(S)::value) < c && ks < key) ? 1u : 0u;
            });
            if (act) {
                place(q + rank, key, nv[q]);
                npos = q + rank;
                nkey = key;
            }
        }
        if (one_run) {
            // slots past a piece's count repeat its last key with an all-ones
            // value: the piece's last element sits on one lane, as an old or
            // a new element; lanes past the count write one slot each
            for (uint32_t j = 0; j < k; ++j) {
                const uint64_t s0 = pstart(j, total, k), s1 = pstart(j + 1, total, k);
                const uint32_t cnt = static_cast<uint32_t>(s1 - s0);
                if (cnt >= static_cast<uint32_t>(kSlots)) continue;
                const uint64_t mo = group_bits<kNodeLanes>(__ballot(opos == s1 - 1), gbase);
                const uint64_t mn = group_bits<kNodeLanes>(__ballot(npos == s1 - 1), gbase);
                const K ko = __shfl(okey, gbase + (mo ? __builtin_ctzll(mo) : 0), 64);
                const K kn = __shfl(nkey, gbase + (mn ? __builtin_ctzll(mn) : 0), 64);
                const K lastk = mo ? ko : kn;
                const uint64_t dest = j == 0 ? leaf : base_new + j - 1;
                if (static_cast<uint32_t>(gl) >= cnt) {
                    t.lkeys[dest * kSlots + gl] = lastk;
                    t.lvals[dest * kSlots + gl] = kmax<K>();
                }
            }
        }
    }
}

// Rebuild the changed parents of level d: kNodeLanes lanes per parent, group
// grp of ngrp.
template <class K>
__device__ __forceinline__ void apply_inner_body(TreeView<K> t, Ins<K> v, int d, uint64_t grp, uint64_t ngrp,
                                                 const ItemView& iv) {
    const uint32_t ok = v.st->ok;
    const int h = static_cast<int>(v.st->height);
    const int l = h - 1 - d;
    // no child at level d-1 split: no parent at level d changes
    if (!ok || l < 0 || v.st->lvl_new[d - 1] == 0) return;
    const uint64_t n = v.st->lvl_count[d];
    const uint32_t bd = v.st->lvl_base[d], bc = v.st->lvl_base[d - 1];
    const uint32_t alloc = v.st->lvl_alloc[d], alloc_c = v.st->lvl_alloc[d - 1];
    const uint32_t psep_d = v.st->lvl_psep[d], psep_c = v.st->lvl_psep[d - 1];
    const bool child_leaf = d == 1;
    const int gl = lane_id() % kNodeLanes, gbase = lane_id() - gl;
    const uint32_t lane = static_cast<uint32_t>(gl);  // this lane's old slot
    for (uint64_t j = grp; j < n; j += ngrp) {
        const uint32_t node = iv.node[bd + j];
        const uint32_t first = iv.first[bd + j], end = iv.end[bd + j];
        const uint32_t C = iv.cold[bd + j];
        const uint32_t P = iv.k[bd + j];
        const uint32_t off = iv.off[bd + j];
        const K osep = t.ikeys[static_cast<uint64_t>(node) * kSlots + lane];
        const uint32_t ochild = t.ichild[static_cast<uint64_t>(node) * kSlots + lane];
        // the child items (one per changed child node, so at most kSlots),
        // one per lane: slot in this node, piece count, first new piece
        const uint32_t nci = end - first < static_cast<uint32_t>(kNodeLanes) ? end - first : kNodeLanes;
        uint32_t ccs = kNone, cks = 1, cof = 0;
        if (lane < nci) {
            ccs = iv.cs[bc + first + lane];
            cks = iv.k[bc + first + lane];
            cof = iv.off[bc + first + lane];
        }
        // per old slot: shift from split children before it, and its own
        // item (lanes past nci hold no item: slot kNone, one piece, so they
        // add nothing; the moves are row broadcasts)
        uint32_t shift = 0, myk = 1, myoff = 0;
        uint32_t a = 0;  // below 2^21: at most 16 children of at most 2^17 pieces
        static_for<0, kNodeLanes>([&](auto S) {
            constexpr int i = decltype(S)::value;
            const uint32_t cs = row_lane<i>(ccs), ki = row_lane<i>(cks), oi = row_lane<i>(cof);
            a += ki - 1;
            if (cs < lane) shift += ki - 1;
            if (cs == lane) { myk = ki; myoff = oi; }
        });
        __threadfence_block();  // the old node is in registers before any write
        if (a == 0) continue;   // no child split: the parent is unchanged
        const uint32_t newpos = lane + shift;
        const uint32_t Cp = C + a;
        const uint32_t base_new = alloc + off;
        for (uint32_t e0 = 0; e0 < Cp; e0 += kNodeLanes) {
            const uint32_t e = e0 + lane;
            const bool act = e < Cp;
            // old slot whose entries cover e: the last slot with newpos <= e
            uint32_t sf = 0;
            static_for<0, kNodeLanes>([&](auto S) {
                constexpr uint32_t s = decltype(S)::value;
                const uint32_t np = row_lane<s>(newpos);
                if (s < C && np <= e) sf = s;
            });
            const int src = gbase + static_cast<int>(sf);
            const uint32_t np = shfl_u32(newpos, src);
            const uint32_t ks = shfl_u32(myk, src);
            const uint32_t ko = shfl_u32(myoff, src);
            const K os = __shfl(osep, src, 64);
            const uint32_t oc = shfl_u32(ochild, src);
            const uint32_t jj = e - np;
            const K last_sep = (sf + 1 < C) ? os : kmax<K>();
            K sep;
            uint32_t ch;
            if (ks <= 1) {
                sep = last_sep;
                ch = oc;
            } else {
                sep = (jj + 1 < ks) ? v.psep[psep_c + ko + jj] : last_sep;
                if (jj == 0) ch = oc;
                else {
                    const uint32_t id = alloc_c + ko + jj - 1;
                    ch = child_leaf ? (kLeafTag | id) : id;
                }
            }
            if (act) {
                const uint32_t pj = ppart(e, Cp, P);
                const uint32_t s0 = pstart(pj, Cp, P), s1 = pstart(pj + 1, Cp, P);
                const uint32_t slot = e - s0;
                const uint32_t cnt = s1 - s0;
                const uint32_t dest = pj == 0 ? node : base_new + pj - 1;
                t.ikeys[static_cast<uint64_t>(dest) * kSlots + slot] = (slot + 1 < cnt) ? sep : kmax<K>();
                t.ichild[static_cast<uint64_t>(dest) * kSlots + slot] = ch;
                if (e + 1 == s1 && pj + 1 < P) v.psep[psep_d + off + pj] = sep;
            }
        }
        // slots past a piece's count: the largest key and no child, one slot
        // per lane
        for (uint32_t pj = 0; pj < P; ++pj) {
            const uint32_t cnt = pstart(pj + 1, Cp, P) - pstart(pj, Cp, P);
            const uint32_t dest = pj == 0 ? node : base_new + pj - 1;
            if (lane >= cnt) {
                t.ikeys[static_cast<uint64_t>(dest) * kSlots + lane] = kmax<K>();
                t.ichild[static_cast<uint64_t>(dest) * kSlots + lane] = kNone;
            }
        }
    }
}

template <class K>
__global__ __launch_bounds__(kBlk) void k_apply_leaves(TreeView<K> t, Ins<K> v) {
    apply_leaves_body<K>(t, v, gtid() / kNodeLanes, gstride() / kNodeLanes, items_in(v));
}

template <class K>
__global__ __launch_bounds__(kBlk) void k_apply_inner(TreeView<K> t, Ins<K> v, int d) {
    apply_inner_body<K>(t, v, d, gtid() / kNodeLanes, gstride() / kNodeLanes, items_in(v));
}

// Root growth: pack the root's pieces into new levels (one workgroup).
template <class K>
__device__ __forceinline__ void grow_body(TreeView<K> t, Ins<K> v) {
    if (!v.st->ok || v.st->grow_levels == 0) return;
    const int h = static_cast<int>(v.st->height);
    const int dr = h - 1;
    const uint32_t item = v.st->lvl_base[dr];
    const uint32_t k0 = v.it_k[item];
    const uint32_t off = v.it_off[item];
    const uint32_t alloc = v.st->lvl_alloc[dr];
    const uint32_t psep0 = v.st->lvl_psep[dr];
    const bool leaf = dr == 0;
    for (uint32_t e = threadIdx.x; e < k0; e += blockDim.x) {
        const uint32_t id = e == 0 ? v.it_node[item] : alloc + off + e - 1;
        v.gid0[e] = leaf ? (kLeafTag | id) : id;
        v.gsep0[e] = (e + 1 < k0) ? v.psep[psep0 + off + e] : kmax<K>();
    }
    __syncthreads();
    K* sa = v.gsep0; K* sb = v.gsep1;
    uint32_t* ia = v.gid0; uint32_t* ib = v.gid1;
    uint64_t cnt = k0;
    uint32_t cursor = v.st->new_root;
    while (cnt > 1) {
        const uint64_t nodes = cnt <= kSlots ? 1 : (cnt + kSlots - 1) / kSlots;
        for (uint64_t e = threadIdx.x; e < cnt; e += blockDim.x) {
            const uint64_t n = part_of(e, cnt, nodes);
            const uint64_t s0 = part_start(n, cnt, nodes), s1 = part_start(n + 1, cnt, nodes);
            const uint64_t slot = e - s0, c = s1 - s0;
            const uint64_t dest = cursor + n;
            t.ikeys[dest * kSlots + slot] = (slot + 1 < c) ? sa[e] : kmax<K>();
            t.ichild[dest * kSlots + slot] = ia[e];
            if (e + 1 == s1) {
                for (uint64_t s = c; s < kSlots; ++s) {
                    t.ikeys[dest * kSlots + s] = kmax<K>();
                    t.ichild[dest * kSlots + s] = kNone;
                }
                sb[n] = sa[e];  // the node's bound is its last entry's separator
                ib[n] = static_cast<uint32_t>(dest);
            }
        }
        __syncthreads();
        cursor += static_cast<uint32_t>(nodes);
        cnt = nodes;
        K* ts = sa; sa = sb; sb = ts;
        uint32_t* ti = ia; ia = ib; ib = ti;
        __syncthreads();
    }
    if (threadIdx.x == 0) v.st->new_root = cursor - 1;
}


template <class K>
__device__ __forceinline__ void ph_commit(TreeView<K> t, Ins<K> v) {
    if (!v.st->ok) return;
    InsState* st = v.st;
    DevHeader* hdr = t.hdr;
    const int h = static_cast<int>(st->height);
    uint32_t inner_new = st->grow_nodes;
    for (int d = 1; d < h; ++d) inner_new += st->lvl_new[d];
    hdr->n_keys += st->R;
    hdr->leaf_used += st->lvl_new[0];
    hdr->inner_used += inner_new;
    if (st->grow_levels) {
        hdr->height = h + st->grow_levels;
        hdr->root = st->new_root;
    }
    hdr->epoch += 1;
    // the mirror (three top inner levels, key count) needs a refresh when the
    // root grew, the tree was empty, or a node of the top three levels was
    // rewritten: parents at tree level l change when their children (item
    // level h-2-l) split
    bool dirty = st->grow_levels > 0 || hdr->n_keys == st->R;
    for (int l = 0; l < 3; ++l) {
        const int dc = h - 2 - l;
        if (dc >= 0 && st->lvl_new[dc] > 0) dirty = true;
    }
    st->mirror_dirty = dirty ? 1u : 0u;
    reinterpret_cast<MirrorHeader*>(t.mirror)->n_keys = hdr->n_keys;
}

// The upper levels of a large batch's plan in one workgroup: from level d0
// on, every level below holds at most kTailMax items (the pool's per-level
// bound), so the phases run back to back with block scans in LDS where the
// lower levels have kernel boundaries and device-wide scans.
constexpr uint32_t kTailMax = 2048;
constexpr int kTailBlock = 1024;

// exclusive scan of in[0..n) (n <= 2 * blockDim.x) into out, total to *tot
__device__ __forceinline__ void tail_scan(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* tot,
                                          uint32_t* sh) {
    const uint32_t i0 = 2 * threadIdx.x, i1 = i0 + 1;
    const uint32_t a = i0 < n ? in[i0] : 0u, b = i1 < n ? in[i1] : 0u;
    uint32_t total;
    const uint32_t off = block_excl_scan<uint32_t>(a + b, sh, &total);
    if (i0 < n) out[i0] = off;
    if (i1 < n) out[i1] = off + a;
    if (threadIdx.x == 0) *tot = total;
    __syncthreads();
}

template <class K>
__global__ __launch_bounds__(kTailBlock) void k_plan_tail(TreeView<K> t, Ins<K> v0, int d0, int H) {
    __shared__ uint32_t sh[33];
    __shared__ uint32_t sf0[kTailMax + 1], sf1[kTailMax + 1];
    Ins<K> v = v0;
    v.f0 = sf0;
    v.f1 = sf1;
    const uint64_t tid = threadIdx.x, nth = blockDim.x;
    const int h = static_cast<int>(v.st->height);
    for (int d = d0; d < H && d < h; ++d) {
        ph_par_heads<K>(v, d, tid, nth);
        __syncthreads();
        tail_scan(v.f0, v.f1, v.st->lvl_count[d - 1], &v.st->lvl_count[d], sh);
        ph_par_items<K>(v, d, tid, nth);
        __syncthreads();
        ph_par_plan<K>(t, v, d, tid, nth);
        __syncthreads();
        tail_scan(v.f0, v.f1, v.st->lvl_count[d], &v.st->lvl_new[d], sh);
        ph_par_off<K>(v, d, tid, nth);
        __syncthreads();
    }
}

// The batch state from device memory into LDS or back, by threads tid of nth
// (a barrier separates the copy from reads of its destination).
__device__ __forceinline__ void copy_state(InsState* dst, const InsState* src, uint32_t tid, uint32_t nth) {
    static_assert(sizeof(InsState) % 4 == 0, "the state copies as words");
    uint32_t* d = reinterpret_cast<uint32_t*>(dst);
    const uint32_t* s = reinterpret_cast<const uint32_t*>(src);
    for (uint32_t i = tid; i < sizeof(InsState) / 4; i += nth) d[i] = s[i];
}

// Orders one wave's LDS accesses around a point (a workgroup barrier where
// the wave works alone).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Everything after the plan for a batch of at most kFusedMax keys, in one
// workgroup: every level has at most that many touched nodes, one round of
// kNodeLanes-lane groups, and barriers stand where the general path has
// kernel boundaries (leaves, each parent level, growth and commit, mirror).
constexpr int kFusedBlock = 1024;
constexpr uint32_t kFusedMax = kFusedBlock / kNodeLanes;  // 64

// every level's items of a batch of at most kFusedMax keys (at most that
// many runs per level)
constexpr uint32_t kFusedItems = kFusedMax * kMaxLevels;

// Besides the items, two things stay on the chip, so that a level waits on
// fewer rounds of device memory:
//  - the batch state (per-level counts, bases, allocation cursors): from
//    device memory each level, the growth and the commit would wait on its
//    fields one read after another;
//  - the separators a level's splits produce (read by the level above and by
//    the root growth): a level adds at most one piece per new key below it,
//    so a batch of at most kFusedMax keys makes at most kFusedItems of them.
template <class K>
__device__ __forceinline__ void ph_small_apply(TreeView<K> t, Ins<K> v0, int H) {
    __shared__ uint32_t s_node[kFusedItems], s_first[kFusedItems], s_end[kFusedItems];
    __shared__ uint32_t s_cold[kFusedItems], s_k[kFusedItems], s_off[kFusedItems];
    __shared__ uint8_t s_cs[kFusedItems];
    __shared__ K s_psep[kFusedItems];
    __shared__ InsState s_st;
    const uint64_t grp = threadIdx.x / kNodeLanes, ngrp = kFusedBlock / kNodeLanes;
    Ins<K> v = v0;
    v.psep = s_psep;
    copy_state(&s_st, v.st, threadIdx.x, blockDim.x);
    // the planned items of every level, copied once: every slot the plan
    // may have written, so that the copy need not wait for the level counts
    // (it and the state arrive in one round of reads)
    const uint32_t span = v.ip_cap < kFusedItems ? static_cast<uint32_t>(v.ip_cap) : kFusedItems;
    for (uint32_t i = threadIdx.x; i < span; i += kFusedBlock) {
        s_node[i] = v.it_node[i];
        s_first[i] = v.it_first[i];
        s_end[i] = v.it_end[i];
        s_cold[i] = v.it_cold[i];
        s_k[i] = v.it_k[i];
        s_off[i] = v.it_off[i];
        s_cs[i] = v.it_cs[i];
    }
    __syncthreads();
    uint32_t total = 0, pieces = 0;
    for (int d = 0; d < H; ++d) {
        const uint32_t e = s_st.lvl_base[d] + s_st.lvl_count[d];
        total = e > total ? e : total;
        pieces += s_st.lvl_new[d];
    }
    if (total > span || pieces > kFusedItems) {  // cannot happen for at most kFusedMax keys
        if (threadIdx.x == 0) atomicOr(&t.hdr->error, kErrInternal);
        return;
    }
    const ItemView iv{s_node, s_first, s_end, s_cold, s_k, s_off, s_cs};
    // every phase below works on the state's copy (the growth and the
    // commit write only fields that no later kernel reads)
    Ins<K> vr = v;
    vr.st = &s_st;
    apply_leaves_body<K>(t, vr, grp, ngrp, iv);
    __syncthreads();
    for (int d = 1; d < H; ++d) {
        if (s_st.lvl_new[d - 1] == 0) break;  // nothing split below: no level above changes
        apply_inner_body<K>(t, vr, d, grp, ngrp, iv);
        __syncthreads();
    }
    grow_body<K>(t, vr);
    __syncthreads();
    if (threadIdx.x == 0) ph_commit<K>(t, vr);
    __syncthreads();
    if (s_st.mirror_dirty) mirror_refresh_body<K, kFusedBlock>(t);
}

template <class K>
__global__ __launch_bounds__(kFusedBlock) void k_small_apply(TreeView<K> t, Ins<K> v, int H) {
    ph_small_apply<K>(t, v, H);
}

// The parent levels from d0 on, the root growth, the commit and the mirror
// in one workgroup: the host starts it at the first level whose item bound
// is at most kTailApplyMax, one round of kNodeLanes-lane groups, so the
// upper levels (and the levels above the tree's current height, which the
// host cannot see) cost no launch each.
constexpr uint32_t kTailApplyMax = kFusedMax;

template <class K>
__global__ __launch_bounds__(kFusedBlock) void k_apply_tail(TreeView<K> t, Ins<K> v, int d0, int H) {
    __shared__ InsState s_st;
    const uint64_t grp = threadIdx.x / kNodeLanes, ngrp = kFusedBlock / kNodeLanes;
    copy_state(&s_st, v.st, threadIdx.x, blockDim.x);
    __syncthreads();
    Ins<K> vr = v;  // the rebuilds read the state's copy
    vr.st = &s_st;
    for (int d = d0; d < H; ++d) {
        if (s_st.lvl_new[d - 1] == 0) break;  // nothing split below: no level above changes
        apply_inner_body<K>(t, vr, d, grp, ngrp, items_in(v));
        __syncthreads();
    }
    grow_body<K>(t, v);
    __syncthreads();
    if (threadIdx.x == 0) ph_commit<K>(t, v);
    __syncthreads();
    if (v.st->mirror_dirty) mirror_refresh_body<K, kFusedBlock>(t);
}

// ------------------------------------------------------ one key (B = 1)
//
// A batch of one key in one workgroup.  Wave 0 descends from the root,
// keeping each inner node's key and child lines (lane s holds slot s, one
// copy per lane in LDS), and finds the key in its leaf.  A present key gets
// its value.  A new key goes into its leaf; a leaf that held 16 keys splits
// evenly into two, and so does every parent, from the leaves up, that held
// 16 children when a child split; a root that splits grows a new root.
// Node ids, separators, padding, the capacity check and the header commit
// are those the batch path (plan, check and apply above) gives a one-key
// batch, so both leave the same tree.  Every read precedes every write; the
// whole workgroup then refreshes the mirror if the top levels changed.
constexpr int kOneBlock = 256;

template <class K>
__global__ __launch_bounds__(kOneBlock) void k_insert_one(TreeView<K> t, const K* __restrict__ keys,
                                                          const K* __restrict__ vals, uint8_t* __restrict__ status) {
    __shared__ K s_sep[kMaxLevels][64];
    __shared__ uint32_t s_ch[kMaxLevels][64];
    __shared__ uint32_t s_node[kMaxLevels], s_cnt[kMaxLevels], s_slot[kMaxLevels];
    __shared__ uint32_t s_dirty;
    const uint32_t tid = threadIdx.x;
    if (tid < 64) {
        const int s = static_cast<int>(tid) & (kSlots - 1);
        const bool w = tid < static_cast<uint32_t>(kSlots);  // the lanes that write slot s
        DevHeader* hdr = t.hdr;
        const K key = keys[0], val = vals[0];
        const uint32_t h = hdr->height, root = hdr->root, err = hdr->error, epoch = hdr->epoch;
        const uint64_t n0 = hdr->n_keys;
        const uint32_t leaf_used = hdr->leaf_used, inner_used = hdr->inner_used;

        // descent: inner level l (0 = root); slot 15 is never a separator
        uint32_t ref = root;
        for (uint32_t l = 0; l + 1 < h; ++l) {
            const uint64_t at = static_cast<uint64_t>(ref) * kSlots + s;
            const K sp = t.ikeys[at];
            const uint32_t c = t.ichild[at];
            const uint32_t ci = static_cast<uint32_t>(__popcll(__ballot(sp < key) & 0x7FFFull));
            const uint32_t cnt =
                1u + static_cast<uint32_t>(__popcll(__ballot(s < kFirstSlot && sp != kmax<K>()) & 0xFFFFull));
            s_sep[l][tid] = sp;
            s_ch[l][tid] = c;
            s_node[l] = ref;
            s_cnt[l] = cnt;
            s_slot[l] = ci;
            ref = shfl_u32(c, static_cast<int>(ci));
        }
        const uint32_t lf = ref & ~kLeafTag;
        const uint64_t la = static_cast<uint64_t>(lf) * kSlots;
        const K lk = t.lkeys[la + s];
        const K lv = t.lvals[la + s];
        const uint2 meta = t.lmeta[lf];
        __threadfence_block();  // every old line is in registers before any write
        const uint64_t eq = __ballot(lk == key) & 0xFFFFull;
        bool ok = !(err & kErrInternal);
        uint32_t dirty = 0;
        if (eq && n0 != 0) {
            // present: the value in place (padding repeats the last key, so
            // the first equal slot is a real one)
            const uint32_t fs = static_cast<uint32_t>(__builtin_ctzll(eq));
            if (tid == 0) {
                status[0] = 1;
                if (ok) {
                    t.lvals[la + fs] = val;
                    hdr->epoch = epoch + 1;
                    reinterpret_cast<MirrorHeader*>(t.mirror)->n_keys = n0;
                }
            }
        } else {
            const uint32_t c = meta.x, total = c + 1;
            const uint32_t pos =
                static_cast<uint32_t>(__popcll(__ballot(static_cast<uint32_t>(s) < c && lk < key) & 0xFFFFull));
            // levels that split, counted from the leaves (0) up
            uint32_t nsplit = total > static_cast<uint32_t>(kSlots) ? 1u : 0u;
            if (nsplit)
                for (int l = static_cast<int>(h) - 2; l >= 0 && s_cnt[l] + 1 > static_cast<uint32_t>(kSlots); --l)
                    ++nsplit;
            const bool grow = nsplit == h;
            const uint32_t leaf_new = nsplit ? 1u : 0u;
            const uint32_t inner_split = nsplit ? nsplit - 1 : 0u;
            const uint32_t inner_new = inner_split + (grow ? 1u : 0u);
            if (static_cast<uint64_t>(leaf_used) + leaf_new > t.leaf_cap ||
                static_cast<uint64_t>(inner_used) + inner_new > t.inner_cap || h + (grow ? 1u : 0u) > kMaxLevels)
                ok = false;
            if (tid == 0) status[0] = 0;
            if (!ok) {
                if (tid == 0 && !(err & kErrInternal)) atomicOr(&hdr->error, kErrCapacity);
            } else {
                // leaf entry e of the c + 1: old keys below pos, the new key,
                // old keys above
                auto lentry = [&](uint32_t e, K& ke, K& ve) {
                    const int src = static_cast<int>(e <= pos ? e : e - 1);
                    const K ok_ = __shfl(lk, src, 64), ov = __shfl(lv, src, 64);
                    ke = e == pos ? key : ok_;
                    ve = e == pos ? val : ov;
                };
                K sepup = K(0);
                uint32_t newref = 0;
                if (total <= static_cast<uint32_t>(kSlots)) {
                    const uint32_t e = static_cast<uint32_t>(s) < total ? static_cast<uint32_t>(s) : total - 1;
                    K ke, ve;
                    lentry(e, ke, ve);
                    if (w) {
                        t.lkeys[la + s] = ke;
                        t.lvals[la + s] = static_cast<uint32_t>(s) < total ? ve : kmax<K>();
                    }
                    if (tid == 0) t.lmeta[lf] = make_uint2(total, meta.y);
                } else {
                    // 17 entries: [0, 8) stay, [8, 17) go to leaf_used
                    const uint64_t nb = static_cast<uint64_t>(leaf_used) * kSlots;
                    K k0, v0, k1, v1, k7, v7;
                    lentry(s < 8 ? static_cast<uint32_t>(s) : 7u, k0, v0);
                    lentry(8u + (s < 9 ? static_cast<uint32_t>(s) : 8u), k1, v1);
                    lentry(7u, k7, v7);
                    if (w) {
                        t.lkeys[la + s] = k0;
                        t.lvals[la + s] = s < 8 ? v0 : kmax<K>();
                        t.lkeys[nb + s] = k1;
                        t.lvals[nb + s] = s < 9 ? v1 : kmax<K>();
                    }
                    if (tid == 0) {
                        t.lmeta[lf] = make_uint2(8u, leaf_used);
                        t.lmeta[leaf_used] = make_uint2(9u, meta.y);
                    }
                    sepup = k7;
                    newref = kLeafTag | leaf_used;
                }
                // parents from the leaf parents up, while a child split
                uint32_t cursor = inner_used;
                bool split = nsplit > 0;
                for (int l = static_cast<int>(h) - 2; l >= 0 && split; --l) {
                    const uint32_t C = s_cnt[l], cs = s_slot[l], node = s_node[l], E = C + 1;
                    const K osp = s_sep[l][tid];
                    const uint32_t och = s_ch[l][tid];
                    // entry e of the C + 1: the split child's slot holds its
                    // first piece with the piece separator, the next entry its
                    // second piece with the child's old separator
                    auto ientry = [&](uint32_t e, K& se, uint32_t& ce) {
                        const uint32_t src = e <= cs ? e : e - 1;
                        const K sv = __shfl(osp, static_cast<int>(src), 64);
                        const uint32_t cv = shfl_u32(och, static_cast<int>(src));
                        se = e == cs ? sepup : (src + 1 < C ? sv : kmax<K>());
                        ce = e == cs + 1 ? newref : cv;
                    };
                    const uint64_t na = static_cast<uint64_t>(node) * kSlots;
                    if (E <= static_cast<uint32_t>(kSlots)) {
                        K se;
                        uint32_t ce;
                        ientry(static_cast<uint32_t>(s) < E ? static_cast<uint32_t>(s) : 0u, se, ce);
                        if (w) {
                            const bool in = static_cast<uint32_t>(s) < E;
                            t.ikeys[na + s] = in && static_cast<uint32_t>(s) + 1 < E ? se : kmax<K>();
                            t.ichild[na + s] = in ? ce : kNone;
                        }
                        split = false;
                    } else {
                        // 17 entries: [0, 8) stay, [8, 17) go to a new node
                        const uint32_t ni = cursor++;
                        const uint64_t nn = static_cast<uint64_t>(ni) * kSlots;
                        K s0, s1, s7;
                        uint32_t c0, c1, c7;
                        ientry(s < 8 ? static_cast<uint32_t>(s) : 0u, s0, c0);
                        ientry(8u + (s < 9 ? static_cast<uint32_t>(s) : 0u), s1, c1);
                        ientry(7u, s7, c7);
                        if (w) {
                            t.ikeys[na + s] = s + 1 < 8 ? s0 : kmax<K>();
                            t.ichild[na + s] = s < 8 ? c0 : kNone;
                            t.ikeys[nn + s] = s + 1 < 9 ? s1 : kmax<K>();
                            t.ichild[nn + s] = s < 9 ? c1 : kNone;
                        }
                        sepup = s7;
                        newref = ni;
                    }
                }
                uint32_t new_root = root;
                if (split) {
                    // the root split: a new root over its two pieces
                    new_root = cursor;
                    const uint32_t oldref = h == 1 ? (kLeafTag | lf) : s_node[0];
                    const uint64_t ra = static_cast<uint64_t>(new_root) * kSlots;
                    if (w) {
                        t.ikeys[ra + s] = s == 0 ? sepup : kmax<K>();
                        t.ichild[ra + s] = s == 0 ? oldref : (s == 1 ? newref : kNone);
                    }
                }
                if (tid == 0) {
                    hdr->n_keys = n0 + 1;
                    hdr->leaf_used = leaf_used + leaf_new;
                    hdr->inner_used = inner_used + inner_new;
                    if (grow) {
                        hdr->height = h + 1;
                        hdr->root = new_root;
                    }
                    hdr->epoch = epoch + 1;
                    reinterpret_cast<MirrorHeader*>(t.mirror)->n_keys = n0 + 1;
                }
                // the mirror's levels change when the tree was empty, the root
                // grew, or children of its top three levels split
                bool d = grow || n0 == 0;
                for (int l = 0; l < 3; ++l) {
                    const int dc = static_cast<int>(h) - 2 - l;
                    if (dc >= 0 && static_cast<uint32_t>(dc) < nsplit) d = true;
                }
                dirty = d ? 1u : 0u;
            }
        }
        if (tid == 0) s_dirty = dirty;
    }
    __syncthreads();
    if (s_dirty) mirror_refresh_body<K, kOneBlock>(t);
}

// The testing switch of the one-key kernel (on by default).
static std::atomic<int> g_single_key{1};
int set_single_key_insert(int on) { return g_single_key.exchange(on ? 1 : 0, std::memory_order_relaxed); }
static bool single_key_insert_on() { return g_single_key.load(std::memory_order_relaxed) != 0; }

// ------------------------------------------------- small batches (B <= 2048)
//
// A rank sort over many workgroups orders the batch and one workgroup
// deduplicates it; after locate, one workgroup sized to the batch plans every
// level (k_small_plan), and up to kFusedMax keys one more workgroup applies
// the whole batch (k_small_apply).  The results are those of the general
// path: the same item arrays and level counters, the same apply bodies.
// Batches of 2 to kFusedMax keys run all of it in one launch by default
// (k_ins_small, below), with the same results.

constexpr uint32_t kSmallInsert = 2048;
static_assert(kSmallInsert <= kRankSortMax, "the small path sorts with rank_sort_small");
constexpr int kSmallBlock = 1024;

// A batch of at most kFusedSortMax keys is ranked here, by the waves that
// hold its keys, each reading the batch from LDS (about B^2 / 16 cycles of
// one CU: cheaper than a launch up to this size); a larger one arrives
// sorted by rank_sort_small, which spreads the comparisons over B / 16 CUs.
constexpr uint32_t kFusedSortMax = 256;

template <class K>
__global__ __launch_bounds__(kSmallBlock) void k_small_prefix(Ins<K> v, const DevHeader* hdr,
                                                               const K* __restrict__ keys, const K* __restrict__ vals,
                                                               uint32_t B, uint8_t* __restrict__ status,
                                                               uint32_t presorted) {
    __shared__ K rk[kSmallInsert];
    __shared__ K sk[kSmallInsert];
    __shared__ uint32_t si[kSmallInsert];
    __shared__ uint32_t sh[33];
    const uint32_t tid = threadIdx.x;
    uint32_t* s = reinterpret_cast<uint32_t*>(v.st);
    for (uint32_t i = tid; i < sizeof(InsState) / 4; i += blockDim.x) s[i] = 0;
    if (presorted) {
        // the pairs in (key, index) order, from rank_sort_small
        for (uint32_t i = tid; i < B; i += blockDim.x) {
            sk[i] = v.sk[i];
            si[i] = v.si[i];
        }
    } else {
        for (uint32_t i = tid; i < B; i += blockDim.x) rk[i] = keys[i];
        __syncthreads();
        // each element's stable rank over the batch in LDS; only the waves
        // that hold elements count (all lanes of a wave read the same word)
        if (tid < B) {
            const K k0 = rk[tid];
            uint32_t c = 0, j = 0;
            for (; j + 8 <= B; j += 8) {
#pragma unroll
                for (uint32_t u = 0; u < 8; ++u) {
                    const K kj = rk[j + u];
                    c += (kj < k0 || (kj == k0 && j + u < tid)) ? 1u : 0u;
                }
            }
            for (; j < B; ++j) c += (rk[j] < k0 || (rk[j] == k0 && j < tid)) ? 1u : 0u;
            sk[c] = k0;
            si[c] = tid;
        }
        __syncthreads();
        for (uint32_t i = tid; i < B; i += blockDim.x) {
            v.sk[i] = sk[i];
            v.si[i] = si[i];  // locate writes each distinct key's status through it
        }
    }
    __syncthreads();  // the pairs in LDS, the batch state cleared
    if (tid == 0) v.st->height = hdr->height;
    uint32_t f[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const uint32_t p = 2 * tid + e;
        f[e] = (p < B && (p == 0 || sk[p] != sk[p - 1])) ? 1u : 0u;
    }
    uint32_t tot;
    const uint32_t off = block_excl_scan<uint32_t>(f[0] + f[1], sh, &tot);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const uint32_t p = 2 * tid + e;
        if (p >= B) continue;
        const uint32_t pos = off + (e ? f[0] : 0u);
        if (f[e]) {
            v.uk[pos] = sk[p];
            v.upos[pos] = p;
        } else {
            status[si[p]] = 1;  // UPDATED: an earlier occurrence exists
        }
        if (p + 1 == B || sk[p + 1] != sk[p]) v.uv[pos + f[e] - 1] = vals[si[p]];
    }
    if (tid == 0) v.st->U = tot;
}

// Old entry count of node `node` at level d (0 = leaves): a leaf's count, or
// the number of child references of an inner node.
template <class K>
__device__ __forceinline__ uint32_t old_count(const TreeView<K>& t, uint32_t node, bool leaf) {
    if (leaf) return t.lmeta[node].x;
    const uint4* ch = reinterpret_cast<const uint4*>(t.ichild + static_cast<uint64_t>(node) * kSlots);
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < kSlots / 4; ++q) {
        const uint4 x = ch[q];
        c += (x.x != kNone) + (x.y != kNone) + (x.z != kNone) + (x.w != kNone);
    }
    return c;
}

// Exclusive scan over the plan's workgroup: one wave needs no LDS.
template <int NT>
__device__ __forceinline__ uint32_t plan_scan(uint32_t x, uint32_t* sh, uint32_t* total) {
    if constexpr (NT == 64) {
        const uint32_t inc = wave_incl_scan(x);
        *total = __shfl(inc, 63, 64);
        return inc - x;
    } else {
        return block_excl_scan<uint32_t>(x, sh, total);
    }
}

// Locate's records of a batch of at most kFusedMax distinct keys, by tree
// level l (0 = the leaves' parents) and key: the parent, its entry count
// and the slot taken, and each key's leaf entry count.  The one-launch
// insert stages them in LDS with all its threads before it plans.
struct PlanRecs {
    uint32_t pn[kMaxLevels][kFusedMax];
    uint8_t pc[kMaxLevels][kFusedMax];
    uint8_t pi[kMaxLevels][kFusedMax];
    uint8_t ulc[kFusedMax];
};

// Plan of a small batch, one workgroup of NT threads (NT >= B / 2); thread t
// owns new keys 2t and 2t+1.  Small NT keeps the barriers cheap (one wave
// for B <= 128), and the level loops stay rolled so that the kernel's code
// stays small (a single wave runs it once, so every instruction line it
// touches is a cache miss).
//
// The nodes a new key passes through are known from the locate kernel (its
// leaf and, at every level, its parent, the parent's size and the slot taken),
// so the items of every level (runs of new keys through one node) are cut
// first, level after level in LDS with block scans, each item taking its
// node's old entry count from those records.  The piece counts then follow
// level after level: an item gains the new keys of its run (leaves) or
// sum(k - 1) over its child items (inner nodes), a difference of the child
// level's piece-offset prefix taken by the run's first and last keys.  Writes
// the same item arrays and level counters as the general path, and then the
// values of keys already present.
template <class K, int NT>
__device__ __forceinline__ void ph_small_plan(TreeView<K> t, Ins<K> v, int H) {
    constexpr int kL = kMaxLevels;
    constexpr uint32_t kCap = 2 * NT;  // new keys, items per level
    __shared__ uint32_t sh[33];
    __shared__ uint32_t s_a[kCap], s_b[kCap];  // key -> distinct key, node; later prefix sums at item bounds
    __shared__ uint16_t s_ix[kL * kCap];       // item index of each key, per level
    __shared__ uint32_t s_k[kCap + 1];         // piece-offset prefix of the previous level's items
    __shared__ uint8_t s_C[kL * kCap];         // old entry count of every item
    __shared__ uint32_t s_base[kL + 1];        // first item of each level
    __shared__ uint32_t s_over;
    __shared__ InsState s_st;  // the batch state, written back at the end
    const uint32_t tid = threadIdx.x;
    copy_state(&s_st, v.st, tid, NT);
    __syncthreads();
    const uint32_t U = s_st.U;
    const int h = static_cast<int>(s_st.height);
    const int hmax = H < h ? H : h;
    if (tid == 0) s_over = 0;

    // new keys in key order (locate left f0[u] = 1 for a key not in its leaf)
    uint32_t fl[2];
    for (int j = 0; j < 2; ++j) {
        const uint32_t u = 2 * tid + j;
        fl[j] = u < U ? v.f0[u] : 0u;
    }
    uint32_t R;
    const uint32_t o0 = plan_scan<NT>(fl[0] + fl[1], sh, &R);
    for (int j = 0; j < 2; ++j) {
        if (!fl[j]) continue;
        const uint32_t u = 2 * tid + j, r = o0 + (j ? fl[0] : 0u);
        const uint32_t leaf = v.uleaf[u];
        v.nk[r] = v.uk[u];
        v.nv[r] = v.uv[u];
        v.nleaf[r] = leaf;
        v.nu[r] = u;
        s_a[r] = u;
        s_b[r] = leaf;
    }
    __syncthreads();
    bool valid[2];
    // per key and level: node, its old entry count and its slot in its
    // parent (all recorded by locate), the next level's loaded one level ahead
    uint32_t nu[2], ixp[2], node[2], cnt[2], cs[2], pnx[2] = {0u, 0u}, pcx[2] = {0u, 0u}, pix[2] = {0u, 0u};
    for (int j = 0; j < 2; ++j) {
        const uint32_t r = 2 * tid + j;
        valid[j] = r < R;
        nu[j] = valid[j] ? s_a[r] : 0u;
        node[j] = valid[j] ? s_b[r] : 0u;
        cnt[j] = valid[j] ? v.ulc[nu[j]] : 0u;
        cs[j] = valid[j] && h >= 2 ? v.pi[static_cast<uint64_t>(h - 2) * v.Bm + nu[j]] : 0u;
        ixp[j] = r;  // at the leaf level an item's range counts keys
    }

    // items of every level: heads and ends of runs, item index per key
    uint32_t hbits = 0, lbits = 0, items = 0;
#pragma unroll 1
    for (int d = 0; d < hmax; ++d) {
        if (d > 0) {
            for (int j = 0; j < 2; ++j) {
                node[j] = pnx[j];
                cnt[j] = pcx[j];
                cs[j] = pix[j];
                if (valid[j]) s_b[2 * tid + j] = node[j];
            }
            __syncthreads();
        }
        // the next level's records, in flight through this level
        if (d + 1 < hmax)
            for (int j = 0; j < 2; ++j) {
                const uint64_t at = static_cast<uint64_t>(h - 2 - d) * v.Bm + nu[j];
                pnx[j] = valid[j] ? v.pn[at] : 0u;
                pcx[j] = valid[j] ? v.pc[at] : 0u;
                pix[j] = valid[j] && h - 3 - d >= 0 ? v.pi[at - v.Bm] : 0u;
            }
        uint32_t hd[2], ls[2];
        for (int j = 0; j < 2; ++j) {
            const uint32_t r = 2 * tid + j;
            hd[j] = valid[j] && (r == 0 || s_b[r - 1] != node[j]) ? 1u : 0u;
            ls[j] = valid[j] && (r + 1 == R || s_b[r + 1] != node[j]) ? 1u : 0u;
        }
        uint32_t n;
        const uint32_t oh = plan_scan<NT>(hd[0] + hd[1], sh, &n);
        for (int j = 0; j < 2; ++j) {
            const uint32_t r = 2 * tid + j;
            const uint32_t ix = oh + (j ? hd[0] : 0u) + hd[j] - 1u;
            const uint64_t e = static_cast<uint64_t>(items) + ix;
            if (valid[j]) s_ix[d * kCap + r] = static_cast<uint16_t>(ix);
            if (hd[j]) {
                if (e < v.ip_cap) {
                    v.it_node[e] = node[j];
                    v.it_rep[e] = nu[j];
                    v.it_first[e] = ixp[j];
                    v.it_cold[e] = cnt[j];
                    v.it_cs[e] = static_cast<uint8_t>(cs[j]);
                    s_C[e] = static_cast<uint8_t>(cnt[j]);
                } else {
                    s_over = 1;
                }
            }
            if (ls[j] && e < v.ip_cap) v.it_end[e] = ixp[j] + 1u;
            hbits |= hd[j] << (2 * d + j);
            lbits |= ls[j] << (2 * d + j);
            ixp[j] = ix;
        }
        if (tid == 0) s_base[d] = items;
        items += n;
        __syncthreads();  // s_b is rewritten by the next level
    }
    if (tid == 0) s_base[hmax] = items;
    __syncthreads();

    const uint32_t total = items < v.ip_cap ? items : static_cast<uint32_t>(v.ip_cap);

    // piece counts, level after level.  An item's gain is its run's key
    // count (leaves) or sum(k - 1) over its child items (inner levels): a
    // difference of the child level's piece-offset prefix (s_k), taken by
    // the run's first and last keys.
    // Every LDS read of a step is issued before any of them is used (the
    // indexes of keys and items past the end are clamped to 0 rather than
    // branched around), and each key's item at the level below stays in a
    // register: a single wave otherwise waits out one LDS round trip per read.
    uint32_t psep = 0;
    uint32_t below[2] = {0u, 0u};  // each key's item index at level d - 1
#pragma unroll 1
    for (int d = 0; d < hmax; ++d) {
        const uint32_t bd = s_base[d], nd = s_base[d + 1] - bd;
        uint32_t ixd[2], c[2], e[2];
        for (int j = 0; j < 2; ++j) {
            const uint32_t r = 2 * tid + j;
            ixd[j] = s_ix[d * kCap + (valid[j] ? r : 0u)];
            c[j] = d == 0 ? r : s_k[below[j]];
            e[j] = d == 0 ? r + 1 : s_k[below[j] + 1];
        }
        for (int j = 0; j < 2; ++j) {
            if (!valid[j]) continue;
            if ((hbits >> (2 * d + j)) & 1u) s_a[ixd[j]] = c[j];
            if ((lbits >> (2 * d + j)) & 1u) s_b[ixd[j]] = e[j];
            below[j] = ixd[j];
        }
        __syncthreads();
        uint32_t kk[2], f[2];
        for (int i = 0; i < 2; ++i) {
            const uint32_t jt = 2 * tid + i;
            const bool in = jt < nd && bd + jt < total;
            const uint32_t at = in ? jt : 0u;
            const uint32_t C = s_C[in ? bd + jt : 0u], hi = s_b[at], lo = s_a[at];
            kk[i] = in ? split_pieces(static_cast<uint64_t>(C) + (hi - lo)) : 1u;
            f[i] = in ? kk[i] - 1u : 0u;
        }
        uint32_t nnew;
        const uint32_t of = plan_scan<NT>(f[0] + f[1], sh, &nnew);
        // s_k now holds this level's piece-offset prefix, s_k[nd] its total
        for (int i = 0; i < 2; ++i) {
            const uint32_t jt = 2 * tid + i;
            const uint32_t o = of + (i ? f[0] : 0u);
            if (jt < nd) s_k[jt] = o;
            if (jt < nd && bd + jt < total) {
                v.it_k[bd + jt] = kk[i];
                v.it_off[bd + jt] = o;
            }
        }
        if (tid == 0) {
            s_k[nd] = nnew;
            s_st.lvl_count[d] = nd;
            s_st.lvl_base[d] = bd;
            s_st.lvl_new[d] = nnew;
            s_st.lvl_psep[d] = psep;
        }
        psep += nnew;
        __syncthreads();
    }
    if (tid == 0) {
        s_st.R = R;
        if (s_over) s_st.overflow = 1;
    }
    __syncthreads();
    // the check reads the level counters one after another: from LDS
    Ins<K> vs = v;
    vs.st = &s_st;
    ph_check<K>(t, vs, tid, NT);
    __syncthreads();
    copy_state(v.st, &s_st, tid, NT);
    // values of keys already present (the batch passed the capacity check;
    // the leaf rewrites that follow read these values)
    // (at most 2 NT distinct keys: each thread's two are read before either
    // is written, so the reads take one round)
    if (s_st.ok) {
        uint32_t found[2], leaf[2], slot[2];
        K val[2];
        for (int j = 0; j < 2; ++j) {
            const uint32_t u = tid + j * NT;
            const bool in = u < U;
            found[j] = in ? v.ufound[u] : 0u;
            leaf[j] = in ? v.uleaf[u] : 0u;
            slot[j] = in ? v.uslot[u] : 0u;
            val[j] = in ? v.uv[u] : K(0);
        }
        for (int j = 0; j < 2; ++j)
            if (found[j]) t.lvals[static_cast<uint64_t>(leaf[j]) * kSlots + slot[j]] = val[j];
    }
}

template <class K, int NT>
__global__ __launch_bounds__(NT) void k_small_plan(TreeView<K> t, Ins<K> v, int H) {
    ph_small_plan<K, NT>(t, v, H);
}

// The plan of a one-launch insert (at most kFusedMax distinct keys, one per
// lane of a wave), by the whole workgroup.  The items of every level are cut
// at once, one wave per level: a level's run heads and each key's item index
// (a wave scan over the heads) depend only on that level's nodes, which
// locate recorded (staged in LDS in `rec`).  The item arrays follow once the
// level bases are known; then one wave takes the piece counts level after
// level (each level's offsets need the level below), the capacity check and
// the values of present keys, as the small path's plan does, with the same
// item arrays and level counters.
template <class K>
__device__ __forceinline__ void ph_fused_plan(TreeView<K> t, Ins<K> v, int H, const PlanRecs& rec) {
    constexpr int kL = kMaxLevels;
    constexpr uint32_t kCap = kFusedMax;
    static_assert(kFusedBlock / 64 >= kL, "a wave per level");
    __shared__ uint32_t s_nu[kCap], s_leaf[kCap];  // new key -> distinct key, leaf
    __shared__ uint8_t s_ix[kL][kCap];              // item index of each new key, per level
    __shared__ uint32_t s_n[kL], s_base[kL + 1];    // items per level, first item of each level
    __shared__ uint32_t s_lo[kCap], s_hi[kCap];     // a level's item bounds in the level below's prefix
    __shared__ uint32_t s_k[kCap + 1];              // piece-offset prefix of the level below
    __shared__ uint8_t s_C[kL * kCap];              // old entry count of every item
    __shared__ uint32_t s_R, s_over;
    __shared__ InsState s_st;                       // the batch state, written back at the end
    const uint32_t tid = threadIdx.x, lane = tid % 64, w = tid / 64;
    copy_state(&s_st, v.st, tid, kFusedBlock);
    __syncthreads();
    const uint32_t U = s_st.U;
    const int h = static_cast<int>(s_st.height);
    const int hmax = H < h ? H : h;

    // new keys in key order (locate left f0[u] = 1 for a key not in its leaf)
    if (w == 0) {
        const uint32_t u = lane;
        const uint32_t f = u < U ? v.f0[u] : 0u;
        const uint32_t inc = wave_incl_scan(f);
        if (f) {
            const uint32_t r = inc - 1u, leaf = v.uleaf[u];
            v.nk[r] = v.uk[u];
            v.nv[r] = v.uv[u];
            v.nleaf[r] = leaf;
            v.nu[r] = u;
            s_nu[r] = u;
            s_leaf[r] = leaf;
        }
        if (lane == 63) {
            s_R = inc;
            s_over = 0;
        }
    }
    __syncthreads();
    const uint32_t R = s_R;

    // each level's items: run heads and ends, item index per key (wave d)
    const int d = static_cast<int>(w);
    const uint32_t r = lane;
    const bool valid = d < hmax && r < R;
    const uint32_t nu = valid ? s_nu[r] : 0u;
    auto node_at = [&](uint32_t x) { return d == 0 ? s_leaf[x] : rec.pn[h - 1 - d][s_nu[x]]; };
    uint32_t node = 0, hd = 0, ls = 0;
    if (valid) {
        node = node_at(r);
        hd = (r == 0 || node_at(r - 1) != node) ? 1u : 0u;
        ls = (r + 1 == R || node_at(r + 1) != node) ? 1u : 0u;
    }
    uint32_t ix = 0;
    if (d < hmax) {
        const uint32_t inc = wave_incl_scan(hd);
        ix = inc - 1u;
        if (valid) s_ix[d][r] = static_cast<uint8_t>(ix);
        if (lane == 63) s_n[d] = inc;
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t items = 0;
        for (int l = 0; l < hmax; ++l) {
            s_base[l] = items;
            items += s_n[l];
        }
        s_base[hmax] = items;
    }
    __syncthreads();
    // the item arrays: node, representative key, range of child items (keys
    // at the leaves), old entry count, slot in the parent
    if (valid) {
        const uint64_t e = static_cast<uint64_t>(s_base[d]) + ix;
        const uint32_t ixp = d == 0 ? r : s_ix[d - 1][r];
        if (hd) {
            if (e < v.ip_cap) {
                const uint32_t cnt = d == 0 ? rec.ulc[nu] : rec.pc[h - 1 - d][nu];
                const uint32_t cs = h - 2 - d >= 0 ? rec.pi[h - 2 - d][nu] : 0u;
                v.it_node[e] = node;
                v.it_rep[e] = nu;
                v.it_first[e] = ixp;
                v.it_cold[e] = cnt;
                v.it_cs[e] = static_cast<uint8_t>(cs);
                s_C[e] = static_cast<uint8_t>(cnt);
            } else {
                s_over = 1;
            }
        }
        if (ls && e < v.ip_cap) v.it_end[e] = ixp + 1u;
    }
    __syncthreads();
    if (w != 0) return;

    // piece counts, level after level (one key and one item per lane): an
    // item gains its run's key count (leaves) or sum(k - 1) over its child
    // items, a difference of the level below's piece-offset prefix taken by
    // the run's first and last keys
    const uint32_t total_items = s_base[hmax];
    const uint32_t total = total_items < v.ip_cap ? total_items : static_cast<uint32_t>(v.ip_cap);
    const bool kv = r < R;
    uint32_t psep = 0, below = 0;
#pragma unroll 1
    for (int l = 0; l < hmax; ++l) {
        const uint32_t bd = s_base[l], nd = s_base[l + 1] - bd;
        const uint32_t ixl = kv ? s_ix[l][r] : 0u;
        const uint32_t lo = l == 0 ? r : s_k[below], hi = l == 0 ? r + 1 : s_k[below + 1];
        const bool head = kv && (r == 0 || s_ix[l][r - 1] != ixl);
        const bool end = kv && (r + 1 == R || s_ix[l][r + 1] != ixl);
        if (head) s_lo[ixl] = lo;
        if (end) s_hi[ixl] = hi;
        below = ixl;
        wave_sync();
        const uint32_t jt = lane;
        const bool in = jt < nd && bd + jt < total;
        const uint32_t C = s_C[in ? bd + jt : 0u], ih = s_hi[in ? jt : 0u], il = s_lo[in ? jt : 0u];
        const uint32_t kk = in ? split_pieces(static_cast<uint64_t>(C) + (ih - il)) : 1u;
        const uint32_t f = in ? kk - 1u : 0u;
        const uint32_t inc = wave_incl_scan(f);
        const uint32_t nnew = __shfl(inc, 63, 64), o = inc - f;
        if (jt < nd) s_k[jt] = o;
        if (in) {
            v.it_k[bd + jt] = kk;
            v.it_off[bd + jt] = o;
        }
        if (lane == 0) {
            s_k[nd] = nnew;
            s_st.lvl_count[l] = nd;
            s_st.lvl_base[l] = bd;
            s_st.lvl_new[l] = nnew;
            s_st.lvl_psep[l] = psep;
        }
        psep += nnew;
        wave_sync();
    }
    if (lane == 0) {
        s_st.R = R;
        if (s_over) s_st.overflow = 1;
    }
    wave_sync();
    Ins<K> vs = v;
    vs.st = &s_st;
    ph_check<K>(t, vs, lane, 64);
    wave_sync();
    copy_state(v.st, &s_st, lane, 64);
    // values of keys already present (one per lane, read before written)
    if (s_st.ok && lane < U && v.ufound[lane])
        t.lvals[static_cast<uint64_t>(v.uleaf[lane]) * kSlots + v.uslot[lane]] = v.uv[lane];
}

// Stable rank of a[i] = k0 among a[0..n) in LDS (by key, then position):
// eight reads in flight at a time, where one at a time waits out every
// read's latency.
template <class K>
__device__ __forceinline__ uint32_t stable_rank(const K* a, uint32_t n, K k0, uint32_t i) {
    uint32_t c = 0, j = 0;
    for (; j + 8 <= n; j += 8) {
        K x[8];
#pragma unroll
        for (uint32_t q = 0; q < 8; ++q) x[q] = a[j + q];
#pragma unroll
        for (uint32_t q = 0; q < 8; ++q) c += (x[q] < k0 || (x[q] == k0 && j + q < i)) ? 1u : 0u;
    }
    for (; j < n; ++j) c += (a[j] < k0 || (a[j] == k0 && j < i)) ? 1u : 0u;
    return c;
}

// A batch of at most kFusedMax keys in one launch: the small path's kernels
// (rank and distinct keys, locate, plan, apply) as phases of one
// kFusedBlock-thread workgroup, with barriers where the small path has
// kernel boundaries.  The batch is ranked in LDS (by key, then by position,
// as the small path ranks it) and planned with the small path's item arrays
// and counters (ph_fused_plan), so the tree it leaves is the small path's.
template <class K>
__global__ __launch_bounds__(kFusedBlock) void k_ins_small(TreeView<K> t, Ins<K> v, const K* __restrict__ keys,
                                                           const K* __restrict__ vals, uint32_t B,
                                                           uint8_t* __restrict__ status, int H) {
    __shared__ K s_rk[kFusedMax];
    __shared__ K s_sk[kFusedMax];
    __shared__ uint32_t s_si[kFusedMax];
    __shared__ uint32_t sh[33];
    const uint32_t tid = threadIdx.x;
    uint32_t* st = reinterpret_cast<uint32_t*>(v.st);
    for (uint32_t i = tid; i < sizeof(InsState) / 4; i += kFusedBlock) st[i] = 0;
    if (tid < B) s_rk[tid] = keys[tid];
    __syncthreads();
    // each key's stable rank in the batch
    if (tid < B) {
        const K k0 = s_rk[tid];
        const uint32_t c = stable_rank(s_rk, B, k0, tid);
        s_sk[c] = k0;
        s_si[c] = tid;
    }
    __syncthreads();
    // the distinct keys, each with the value of its last occurrence; a
    // repeat reports UPDATED (an earlier occurrence inserts the key)
    const bool in = tid < B;
    const bool head = in && (tid == 0 || s_sk[tid] != s_sk[tid - 1]);
    const bool last = in && (tid + 1 == B || s_sk[tid + 1] != s_sk[tid]);
    if (in) {
        v.sk[tid] = s_sk[tid];
        v.si[tid] = s_si[tid];  // locate writes each distinct key's status through it
        if (!head) status[s_si[tid]] = 1;
    }
    uint32_t U;
    const uint32_t pos = block_excl_scan<uint32_t>(head ? 1u : 0u, sh, &U);
    if (head) {
        v.uk[pos] = s_sk[tid];
        v.upos[pos] = tid;
    }
    if (last) v.uv[pos + (head ? 1u : 0u) - 1u] = vals[s_si[tid]];
    if (tid == 0) {
        v.st->U = U;
        v.st->height = t.hdr->height;
    }
    __syncthreads();
    ph_locate<K, 16, 1, 2, kFusedBlock>(t, v, status);
    __syncthreads();
    // the plan's reads of locate's records, in one round by every thread
    __shared__ PlanRecs s_rec;
    {
        const uint32_t h = v.st->height, Ud = v.st->U;
        const uint32_t nl = h >= 2 ? h - 1 : 0;  // levels 0 .. h-2
        for (uint32_t i = tid; i < nl * Ud; i += kFusedBlock) {
            const uint32_t l = i / Ud, u = i % Ud;
            const uint64_t at = static_cast<uint64_t>(l) * v.Bm + u;
            s_rec.pn[l][u] = v.pn[at];
            s_rec.pc[l][u] = v.pc[at];
            s_rec.pi[l][u] = v.pi[at];
        }
        if (tid < Ud) s_rec.ulc[tid] = v.ulc[tid];
    }
    __syncthreads();
    ph_fused_plan<K>(t, v, H, s_rec);
    __syncthreads();
    ph_small_apply<K>(t, v, H);
}

static std::atomic<int> g_one_launch_insert{1};
int set_one_launch_insert(int on) { return g_one_launch_insert.exchange(on ? 1 : 0, std::memory_order_relaxed); }
static bool one_launch_insert_on() { return g_one_launch_insert.load(std::memory_order_relaxed) != 0; }

// ------------------------------------------------------------------ launch

static uint32_t grid_for(uint64_t n, uint32_t per_block) {
    uint64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return static_cast<uint32_t>(g);
}

template <class K, int G, int QPG, int LV>
static void launch_locate_t(const TreeView<K>& t, const Ins<K>& v, uint64_t B, uint8_t* status, hipStream_t s) {
    const uint32_t lds = LV > 0 ? MirrorLayout<K>::bytes(mirror_nodes_for_levels(LV)) : 0;
    uint32_t grid = grid_for((B + QPG - 1) / QPG, kBlk / G);
    if (grid > 2048) grid = 2048;
    hipLaunchKernelGGL((k_locate<K, G, QPG, LV>), dim3(grid), dim3(kBlk), lds, s, t, v, status);
}

// Shape by batch size, as for lookups: small batches are latency-bound (16
// lanes, one key per group); large ones are bound by the rate of line
// requests (8 lanes, four keys in flight per group).
template <class K, int G, int QPG>
static void launch_locate_lv(const TreeView<K>& t, const Ins<K>& v, const LaunchCfg& cfg, uint64_t B,
                             uint8_t* status, hipStream_t s) {
    switch (cfg.lds_levels) {
        case 0: launch_locate_t<K, G, QPG, 0>(t, v, B, status, s); break;
        case 1: launch_locate_t<K, G, QPG, 1>(t, v, B, status, s); break;
        case 3: launch_locate_t<K, G, QPG, 3>(t, v, B, status, s); break;
        default: launch_locate_t<K, G, QPG, 2>(t, v, B, status, s); break;
    }
}

template <class K>
static void launch_locate(const TreeView<K>& t, const Ins<K>& v, const LaunchCfg& cfg, uint64_t B, uint8_t* status,
                          hipStream_t s) {
    if (B >= kLargeBatch) launch_locate_lv<K, 8, 4>(t, v, cfg, B, status, s);
    else launch_locate_lv<K, 16, 1>(t, v, cfg, B, status, s);
}

// highest tree height the pools allow (non-root inner nodes have >= 8
// children, the root >= 2)
static int height_bound(uint64_t leaf_cap) {
    int h = 1;
    uint64_t cover = 2;  // leaves a tree of height h+1 can have at least
    while (cover <= leaf_cap && h < kMaxLevels - 1) {
        ++h;
        cover *= 8;
    }
    return h + 1 < kMaxLevels ? h + 1 : kMaxLevels;
}

// apply, grow, commit, mirror: shared by both paths (the small path's plan
// kernel writes the updates itself)
template <class K>
static void launch_apply(const TreeView<K>& t, const Ins<K>& v, uint64_t B, uint64_t leaf_cap, int H, bool updates,
                         hipStream_t s) {
    const uint32_t gB = grid_for(B, kBlk);
    if (updates) hipLaunchKernelGGL(k_apply_updates<K>, dim3(gB), dim3(kBlk), 0, s, t, v);
    hipLaunchKernelGGL(k_apply_leaves<K>, dim3(grid_for(B, kBlk / kNodeLanes)), dim3(kBlk), 0, s, t, v);
    int d0 = 1;
    while (d0 < H && level_items_bound(B, leaf_cap, d0) > kTailApplyMax) ++d0;
    for (int d = 1; d < d0; ++d)
        hipLaunchKernelGGL(k_apply_inner<K>, dim3(grid_for(B, kBlk / kNodeLanes)), dim3(kBlk), 0, s, t, v, d);
    hipLaunchKernelGGL(k_apply_tail<K>, dim3(1), dim3(kFusedBlock), 0, s, t, v, d0, H);
}

template <class K>
void launch_insert(const TreeView<K>& t, const InsertCtx& c, const K* keys, const K* vals, uint64_t B,
                   uint8_t* status, hipStream_t s) {
    Ins<K> v;
    carve<K>(&v, c.scratch, c.max_batch, c.leaf_cap, c.inner_cap);
    InsState* st = v.st;
    const uint32_t gB = grid_for(B, kBlk);
    const int H = height_bound(c.leaf_cap);

    if (B == 1 && single_key_insert_on()) {
        hipLaunchKernelGGL(k_insert_one<K>, dim3(1), dim3(kOneBlock), 0, s, t, keys, vals, status);
        return;
    }
    if (B <= kFusedMax && one_launch_insert_on()) {
        const uint32_t lds = MirrorLayout<K>::bytes(mirror_nodes_for_levels(2));
        hipLaunchKernelGGL(k_ins_small<K>, dim3(1), dim3(kFusedBlock), lds, s, t, v, keys, vals,
                           static_cast<uint32_t>(B), status, H);
        return;
    }
    if (B <= kSmallInsert) {
        const uint32_t presorted = B > kFusedSortMax ? 1u : 0u;
        if (presorted) rank_sort_small<K>(keys, static_cast<uint32_t>(B), v.sk, v.si, nullptr, 0, s);
        hipLaunchKernelGGL(k_small_prefix<K>, dim3(1), dim3(kSmallBlock), 0, s, v, t.hdr, keys, vals,
                           static_cast<uint32_t>(B), status, presorted);
        launch_locate<K>(t, v, c.cfg, B, status, s);
        if (B <= 128) hipLaunchKernelGGL((k_small_plan<K, 64>), dim3(1), dim3(64), 0, s, t, v, H);
        else if (B <= 512) hipLaunchKernelGGL((k_small_plan<K, 256>), dim3(1), dim3(256), 0, s, t, v, H);
        else hipLaunchKernelGGL((k_small_plan<K, kSmallBlock>), dim3(1), dim3(kSmallBlock), 0, s, t, v, H);
        if (B <= kFusedMax) hipLaunchKernelGGL(k_small_apply<K>, dim3(1), dim3(kFusedBlock), 0, s, t, v, H);
        else launch_apply<K>(t, v, B, c.leaf_cap, H, false, s);  // the plan wrote the updates
        return;
    }
    hipLaunchKernelGGL(k_init<K>, dim3(1), dim3(kBlk), 0, s, v, t.hdr);
    sort_from<K>(keys, v.sk, v.si, v.sk2, v.si2, B, v.sort_tmp, s, &t.hdr->error, kErrInternal);
    hipLaunchKernelGGL(k_heads<K>, dim3(gB), dim3(kBlk), 0, s, v, B, status);
    scan_exclusive<uint32_t>(v.f0, v.f1, &st->U, nullptr, B, v.scan_tmp, s);
    hipLaunchKernelGGL(k_unique<K>, dim3(gB), dim3(kBlk), 0, s, v, B, vals);
    launch_locate<K>(t, v, c.cfg, B, status, s);
    scan_exclusive<uint32_t>(v.f0, v.f1, &st->R, &st->U, B, v.scan_tmp, s);
    hipLaunchKernelGGL(k_compact_new<K>, dim3(gB), dim3(kBlk), 0, s, v);
    hipLaunchKernelGGL(k_leaf_heads<K>, dim3(gB), dim3(kBlk), 0, s, v);
    scan_exclusive<uint32_t>(v.f0, v.f1, &st->lvl_count[0], &st->R, B, v.scan_tmp, s);
    hipLaunchKernelGGL(k_leaf_items<K>, dim3(gB), dim3(kBlk), 0, s, v);
    hipLaunchKernelGGL(k_leaf_plan<K>, dim3(gB), dim3(kBlk), 0, s, t, v);
    scan_exclusive<uint32_t>(v.f0, v.it_off, &st->lvl_new[0], &st->lvl_count[0], B, v.scan_tmp, s);
    // lower levels: kernels sized by the level's bound; from d0 on (the
    // level below holds at most kTailMax items) one workgroup plans the rest
    int d0 = 1;
    while (d0 < H && level_items_bound(B, c.leaf_cap, d0 - 1) > kTailMax) ++d0;
    for (int d = 1; d < d0; ++d) {
        const uint64_t nb = level_items_bound(B, c.leaf_cap, d - 1), nd = level_items_bound(B, c.leaf_cap, d);
        const uint32_t gb = grid_for(nb, kBlk), gd = grid_for(nd, kBlk);
        hipLaunchKernelGGL(k_par_heads<K>, dim3(gb), dim3(kBlk), 0, s, v, d);
        scan_exclusive<uint32_t>(v.f0, v.f1, &st->lvl_count[d], &st->lvl_count[d - 1], nb, v.scan_tmp, s);
        hipLaunchKernelGGL(k_par_items<K>, dim3(gb), dim3(kBlk), 0, s, v, d);
        hipLaunchKernelGGL(k_par_plan<K>, dim3(gd), dim3(kBlk), 0, s, t, v, d);
        scan_exclusive<uint32_t>(v.f0, v.f1, &st->lvl_new[d], &st->lvl_count[d], nd, v.scan_tmp, s);
        hipLaunchKernelGGL(k_par_off<K>, dim3(gd), dim3(kBlk), 0, s, v, d);
    }
    if (d0 < H) hipLaunchKernelGGL(k_plan_tail<K>, dim3(1), dim3(kTailBlock), 0, s, t, v, d0, H);
    hipLaunchKernelGGL(k_check<K>, dim3(1), dim3(64), 0, s, t, v);
    launch_apply<K>(t, v, B, c.leaf_cap, H, true, s);
}

template void launch_insert<uint32_t>(const TreeView<uint32_t>&, const InsertCtx&, const uint32_t*,
                                      const uint32_t*, uint64_t, uint8_t*, hipStream_t);
template void launch_insert<uint64_t>(const TreeView<uint64_t>&, const InsertCtx&, const uint64_t*,
                                      const uint64_t*, uint64_t, uint8_t*, hipStream_t);

// ---------------------------------------------------------------- delete
//
// A delete batch (Section III: every node but the root stays at least half
// full) shares the insert's front end: sort, distinct keys, and a locate
// that records each key's path.  Then:
//  1. one thread per touched leaf removes the batch's keys from it in place
//     (survivors moved down, padding rewritten).  If the leaf's largest key
//     went and the leaf stays at least half full, it rewrites the separator
//     that holds that key: on the path, the first node whose child slot is
//     not its last;
//  2. one wave per leaf parent with a child left below half full gathers the
//     parent's keys (at most 16 x 16) and spreads them evenly over
//     max(8, ceil(T / 16)) of its leaves, which borrows and merges in one
//     step.  The leaves no longer needed are cleared (count 0) and dropped
//     from the chain, the parent's line is rewritten, and its new largest
//     key goes into its own separator further up.  A parent that is the
//     root keeps at least two leaves, or becomes the single leaf root when
//     16 keys or fewer remain (the root shrinks);
//  3. a parent that would keep fewer than 64 keys would itself fall below
//     half full; the batch flags it and the host rebuilds the tree from its
//     keys.

constexpr uint32_t kHalf = kSlots / 2;

// A counter that earlier threads raised with atomics (in the L2), read past
// the L1, which may still hold its line from before.
__device__ __forceinline__ uint32_t counter(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Inner nodes at depth < kMirrorDepth (0 = the root) are copied in the
// top-levels mirror: rewriting one, or moving the root, means the mirror
// must be refreshed at the commit (otherwise only its key count changes).
constexpr int kMirrorDepth = 3;

template <class K>
__device__ __forceinline__ void note_inner_write(const Ins<K>& v, int depth) {
    if (depth < kMirrorDepth) v.st->mirror_dirty = 1u;
}
constexpr uint64_t kDelListScan = 16384;  // above: the merge list comes from a scan, in key order

template <class K>
__global__ void k_del_heads(Ins<K> v, uint64_t B, uint8_t* __restrict__ status) {
    for (uint64_t p = gtid(); p < B; p += gstride()) {
        const bool head = p == 0 || v.sk[p] != v.sk[p - 1];
        v.f0[p] = head ? 1u : 0u;
        if (!head) status[v.si[p]] = 0;  // ABSENT: an earlier occurrence deleted it
    }
}

template <class K>
__global__ void k_del_unique(Ins<K> v, uint64_t B) {
    for (uint64_t p = gtid(); p < B; p += gstride()) {
        if (v.f0[p]) {
            v.uk[v.f1[p]] = v.sk[p];
            v.upos[v.f1[p]] = static_cast<uint32_t>(p);
        }
    }
}

// Batches up to 2048 keys (after the rank sort, which also cleared the
// batch state): one workgroup, two sorted positions per thread, finds the
// distinct keys, writes the statuses of repeats and the batch state.
template <class K>
__global__ __launch_bounds__(1024) void k_del_small_prefix(Ins<K> v, const DevHeader* hdr, uint32_t B,
                                                           uint8_t* __restrict__ status) {
    __shared__ uint32_t sh[33];
    const uint32_t t = threadIdx.x, p0 = 2 * t, p1 = p0 + 1;
    const bool h0 = p0 < B && (p0 == 0 || v.sk[p0] != v.sk[p0 - 1]);
    const bool h1 = p1 < B && v.sk[p1] != v.sk[p0];
    if (p0 < B && !h0) status[v.si[p0]] = 0;  // ABSENT: an earlier occurrence deleted it
    if (p1 < B && !h1) status[v.si[p1]] = 0;
    uint32_t tot;
    const uint32_t base = block_excl_scan<uint32_t>((h0 ? 1u : 0u) + (h1 ? 1u : 0u), sh, &tot);
    if (h0) {
        v.uk[base] = v.sk[p0];
        v.upos[base] = p0;
    }
    if (h1) {
        const uint32_t e = base + (h0 ? 1u : 0u);
        v.uk[e] = v.sk[p1];
        v.upos[e] = p1;
    }
    if (t == 0) {
        v.st->U = tot;
        v.st->height = hdr->height;
    }
}

// first distinct key of its leaf's run (keys are sorted, so a leaf's keys
// are consecutive)
template <class K>
__device__ __forceinline__ bool leaf_run_head(const Ins<K>& v, uint64_t u) {
    return u == 0 || v.uleaf[u - 1] != v.uleaf[u];
}

// 16 lanes per touched leaf, lane s on slot s: the lanes read the run's
// distinct keys 16 at a time for the slots to remove, then move the kept
// pairs down (new slot = kept slots below) and pad the rest.  The deleted
// count is added once per wave at the end (one atomic per leaf on a single
// address would serialise); k_del_list then lists the leaves left below
// half full, one thread per distinct key.
template <class K>
__device__ __forceinline__ void ph_del_leaf(TreeView<K> t, Ins<K> v) {
    if (t.hdr->error & kErrInternal) return;  // e.g. the batch's device sort gave up
    const uint64_t U = v.st->U;
    const int h = static_cast<int>(v.st->height);
    const int lane = static_cast<int>(threadIdx.x) & 63, s = lane & (kSlots - 1), gbase = lane - s;
    const uint64_t g0 = gtid() / kSlots, gs = gstride() / kSlots;
    uint32_t del = 0;  // keys this group removed (lane 0 of the group)
    for (uint64_t u = g0;; u += gs) {
        if (__ballot(u < U) == 0) break;  // the wave's four groups are done
        const bool head = u < U && leaf_run_head(v, u);  // the same for the group's 16 lanes
        if (u < U && s == 0) v.nu[u] = 0u;  // set to 1 below for a run left below half full
        if (head) {
            const uint32_t leaf = v.uleaf[u];
            uint32_t gone = 0, nd = 0;
            for (uint64_t e0 = u;; e0 += kSlots) {
                const uint64_t e = e0 + static_cast<uint64_t>(s);
                const bool in = e < U && v.uleaf[e] == leaf;
                const bool hit = in && v.ufound[e];
                uint32_t bit = hit ? (1u << v.uslot[e]) : 0u;
                bit |= __shfl_xor(bit, 1);
                bit |= __shfl_xor(bit, 2);
                bit |= __shfl_xor(bit, 4);
                bit |= __shfl_xor(bit, 8);
                gone |= bit;
                nd += static_cast<uint32_t>(__popcll((__ballot(hit) >> gbase) & 0xFFFFull));
                if (((__ballot(in) >> gbase) & 0xFFFFull) != 0xFFFFull) break;  // the run ended in this round
            }
            const uint32_t c = t.lmeta[leaf].x;
            const uint32_t w = c - nd;
            const bool under = h > 1 && w < kHalf;
            if (s == 0) {
                v.f0[u] = under ? 1u : 0u;
                v.nu[u] = under ? 1u : 0u;
            }
            if (nd) {
                K* kl = t.lkeys + static_cast<uint64_t>(leaf) * kSlots;
                K* vl = t.lvals + static_cast<uint64_t>(leaf) * kSlots;
                const K key = kl[s], val = vl[s];
                const bool keep = static_cast<uint32_t>(s) < c && !((gone >> s) & 1u);
                const uint32_t km = static_cast<uint32_t>((__ballot(keep) >> gbase) & 0xFFFFull);
                const uint32_t at = static_cast<uint32_t>(__popc(km & ((1u << s) - 1u)));
                // the new largest key: from the highest kept slot
                const int top = km ? 31 - __clz(km) : 0;
                const K pk = km ? static_cast<K>(__shfl(key, gbase + top, 64)) : kmax<K>();
                if (keep) {
                    kl[at] = key;
                    vl[at] = val;
                }
                if (static_cast<uint32_t>(s) >= w) {
                    kl[s] = pk;
                    vl[s] = kmax<K>();
                }
                if (s == 0) {
                    t.lmeta[leaf].x = w;
                    del += nd;
                    if (!under && w > 0 && ((gone >> (c - 1)) & 1u)) {
                        for (int l = h - 2; l >= 0; --l) {
                            const uint64_t o2 = static_cast<uint64_t>(l) * v.Bm + u;
                            if (v.pi[o2] + 1u < v.pc[o2]) {
                                t.ikeys[static_cast<uint64_t>(v.pn[o2]) * kSlots + v.pi[o2]] = pk;
                                note_inner_write(v, l);
                                break;
                            }
                        }
                    }
                }
            }
        }
    }
    // one add per wave
    for (int o = 32; o > 0; o >>= 1) del += static_cast<uint32_t>(__shfl_xor(static_cast<int>(del), o));
    if (lane == 0 && del) atomicAdd(&v.st->deleted, del);
}

template <class K>
__global__ __launch_bounds__(kBlk) void k_del_leaf(TreeView<K> t, Ins<K> v) {
    ph_del_leaf<K>(t, v);
}

// The leaf runs left below half full, listed for the merge pass: small
// batches append with an atomic (any order); large ones place each run at
// its prefix-scan position, so the list is in key order.
template <class K>
__device__ __forceinline__ void ph_del_list(TreeView<K> t, Ins<K> v) {
    if (t.hdr->error & kErrInternal) return;
    const uint64_t U = v.st->U;
    for (uint64_t u = gtid(); u < U; u += gstride())
        if (v.nu[u]) v.f1[atomicAdd(&v.st->merges, 1u)] = static_cast<uint32_t>(u);
}

template <class K>
__global__ void k_del_list(TreeView<K> t, Ins<K> v) {
    ph_del_list<K>(t, v);
}

template <class K>
__global__ void k_del_list_ordered(TreeView<K> t, Ins<K> v) {
    if (t.hdr->error & kErrInternal) return;
    const uint64_t U = v.st->U;
    for (uint64_t u = gtid(); u < U; u += gstride())
        if (v.nu[u]) v.f1[v.nleaf[u]] = static_cast<uint32_t>(u);
}

// A wave's LDS for merging one listed parent.
template <class K>
struct MergeLds {
    K mk[kSlots * kSlots];
    K mv[kSlots * kSlots];
    uint32_t kid[kSlots], cnt[kSlots], pre[kSlots + 1];
    uint32_t next;
};

// Orders a wave's LDS writes before its lanes' later reads (a wave-level
// barrier: the body runs in one wave).
// One wave per listed parent: wave w of nw takes list entries w, w + nw, ...
// with its own LDS slice (the batch kernel: one wave per workgroup; the
// one-launch delete: the waves of its workgroup).
template <class K>
__device__ __forceinline__ void ph_del_merge(TreeView<K> t, Ins<K> v, bool ordered, uint32_t w, uint32_t nw,
                                             MergeLds<K>& sm) {
    if (t.hdr->error & kErrInternal) return;
    const int h = static_cast<int>(v.st->height);
    if (h < 2) return;
    K* const mk = sm.mk;
    K* const mv = sm.mv;
    uint32_t* const kid = sm.kid;
    uint32_t* const cnt = sm.cnt;
    uint32_t* const pre = sm.pre;
    uint32_t& s_next = sm.next;
    const int lane = lane_id();
    const uint64_t lp = static_cast<uint64_t>(h - 2) * v.Bm;  // path level of the leaves' parents
    const uint32_t nlist = counter(&v.st->merges);
    for (uint32_t li = w; li < nlist; li += nw) {
        // a leaf run that left its leaf below half full; the first such run
        // under its parent merges that parent
        const uint64_t u = v.f1[li];
        const uint32_t P = v.pn[lp + u];
        bool first = true;
        if (ordered) {
            // the list is in key order, and a parent's runs are consecutive
            first = li == 0 || v.pn[lp + v.f1[li - 1]] != P;
        } else {
            for (uint64_t e = u; e-- > 0 && v.pn[lp + e] == P;) {
                if (leaf_run_head(v, e) && v.f0[e]) {
                    first = false;
                    break;
                }
            }
        }
        if (!first) continue;
        const uint32_t nc = v.pc[lp + u];
        const K fs = t.ikeys[static_cast<uint64_t>(P) * kSlots + kFirstSlot];
        if (lane < kSlots) {
            uint32_t ref = kNone;
            if (static_cast<uint32_t>(lane) < nc)
                ref = fs != kmax<K>() ? static_cast<uint32_t>(fs) + static_cast<uint32_t>(lane)
                                      : t.ichild[static_cast<uint64_t>(P) * kSlots + lane];
            kid[lane] = ref & ~kLeafTag;
            const uint32_t c = static_cast<uint32_t>(lane) < nc ? t.lmeta[ref & ~kLeafTag].x : 0u;
            cnt[lane] = c < kSlots ? c : kSlots;
        }
        wave_sync();
        if (lane == 0) {
            uint32_t a = 0;
            for (int i = 0; i < kSlots; ++i) {
                pre[i] = a;
                a += cnt[i];
            }
            pre[kSlots] = a;
            s_next = t.lmeta[kid[nc - 1]].y;
        }
        wave_sync();
        const uint32_t T = pre[kSlots];
        const bool root = h == 2;
        if (!root && T < kHalf * kHalf) {
            // the parent would fall below half full: its grandparent merges
            // it with its siblings (marked 2, listed for the next kernel)
            if (lane == 0) {
                v.f0[u] = 2u;
                v.upos[atomicAdd(&v.st->gmerges, 1u)] = static_cast<uint32_t>(u);
            }
            wave_sync();
            continue;
        }
        {
            // 16 lanes per child, slot = lane % 16, four children per round:
            // every load of the gather in flight at once, few registers
            const uint32_t j = static_cast<uint32_t>(lane) % kSlots;
            K kk[4], vv[4];
#pragma unroll
            for (uint32_t r = 0; r < 4; ++r) {
                const uint32_t c = r * 4 + static_cast<uint32_t>(lane) / kSlots;
                if (c < nc && j < cnt[c]) {
                    kk[r] = t.lkeys[static_cast<uint64_t>(kid[c]) * kSlots + j];
                    vv[r] = t.lvals[static_cast<uint64_t>(kid[c]) * kSlots + j];
                }
            }
#pragma unroll
            for (uint32_t r = 0; r < 4; ++r) {
                const uint32_t c = r * 4 + static_cast<uint32_t>(lane) / kSlots;
                if (c < nc && j < cnt[c]) {
                    mk[pre[c] + j] = kk[r];
                    mv[pre[c] + j] = vv[r];
                }
            }
        }
        wave_sync();
        const uint32_t want = (T + kSlots - 1) / kSlots;
        const uint32_t n0 = root ? (T <= kSlots ? 1u : (want > 2u ? want : 2u)) : (want > kHalf ? want : kHalf);
        if (n0 > nc) {  // cannot happen on a tree whose nodes were at least half full
            if (lane == 0) atomicOr(&v.st->rebuild, 1u);
            wave_sync();
            continue;
        }
        const uint32_t q = T / n0, r = T % n0;
        // leaf j (lane j < n0) takes pairs [start, start + len)
        if (static_cast<uint32_t>(lane) < nc) {
            const uint32_t j = static_cast<uint32_t>(lane);
            const uint64_t dst = static_cast<uint64_t>(kid[j]) * kSlots;
            if (j < n0) {
                const uint32_t len = q + (j < r ? 1u : 0u), start = j * q + (j < r ? j : r);
                for (uint32_t s = 0; s < kSlots; ++s) {
                    t.lkeys[dst + s] = s < len ? mk[start + s] : (len ? mk[start + len - 1] : kmax<K>());
                    t.lvals[dst + s] = s < len ? mv[start + s] : kmax<K>();
                }
                t.lmeta[kid[j]] = make_uint2(len, j + 1 < n0 ? kid[j + 1] : s_next);
            } else {
                for (uint32_t s = 0; s < kSlots; ++s) {
                    t.lkeys[dst + s] = kmax<K>();
                    t.lvals[dst + s] = kmax<K>();
                }
                t.lmeta[kid[j]] = make_uint2(0u, kNone);
            }
        }
        if (lane == 0) note_inner_write(v, h - 2);  // P, or the root it replaces
        if (root && n0 == 1) {
            // the root shrinks to its first leaf
            if (lane == 0) {
                t.hdr->root = kid[0] | kLeafTag;
                t.hdr->height = 1;
            }
        } else {
            if (lane < kSlots) {
                const uint32_t s = static_cast<uint32_t>(lane);
                K sep = kmax<K>();
                if (s + 1 < n0) {
                    const uint32_t end = (s + 1) * q + (s + 1 < r ? s + 1 : r);  // start of leaf s + 1
                    sep = mk[end - 1];
                }
                t.ikeys[static_cast<uint64_t>(P) * kSlots + s] = sep;  // slot 15: children from the child line
                t.ichild[static_cast<uint64_t>(P) * kSlots + s] = s < n0 ? (kid[s] | kLeafTag) : kNone;
            }
            if (lane == 0 && !root) {
                const K top = mk[T - 1];
                for (int l = h - 3; l >= 0; --l) {
                    const uint64_t o2 = static_cast<uint64_t>(l) * v.Bm + u;
                    if (v.pi[o2] + 1u < v.pc[o2]) {
                        t.ikeys[static_cast<uint64_t>(v.pn[o2]) * kSlots + v.pi[o2]] = top;
                        note_inner_write(v, l);
                        break;
                    }
                }
            }
        }
        wave_sync();
    }
}

template <class K>
__global__ __launch_bounds__(64) void k_del_merge(TreeView<K> t, Ins<K> v, bool ordered) {
    __shared__ MergeLds<K> sm;
    ph_del_merge<K>(t, v, ordered, blockIdx.x, gridDim.x, sm);
}

// One level up: a leaf parent that would fall below half full (fewer than
// 64 keys) is merged with its siblings.  One workgroup per grandparent G
// gathers every pair below G (at most 16 x 16 x 16) in LDS and lays them out
// again over n1 = max(8, ceil(T / 256)) of G's parents and
// n0 = max(8 n1, ceil(T / 16)) of its leaves, reusing old ids in key order
// (a subtree that was at least half full has enough of both).  A root G
// keeps at least two parents, or the tree loses levels: one parent as root
// at T <= 256, one leaf at T <= 16.  A G left with fewer than 512 keys would
// itself fall below half full; the host rebuilds the tree instead.
constexpr int kBelowG = kSlots * kSlots * kSlots;

template <class K>
__device__ __forceinline__ void ph_del_merge2(TreeView<K> t, Ins<K> v) {
    if (t.hdr->error & kErrInternal) return;
    const int h = static_cast<int>(v.st->height);
    if (h < 3) return;
    __shared__ K mk[kBelowG];
    __shared__ K mv[kBelowG];
    __shared__ uint32_t lid[kSlots * kSlots];  // G's leaves in key order
    __shared__ uint32_t pid[kSlots];           // G's parents in order
    __shared__ uint32_t sh[33];
    __shared__ uint32_t s_first, s_next;
    const int tid = static_cast<int>(threadIdx.x);
    const uint64_t lg = static_cast<uint64_t>(h - 3) * v.Bm;  // path level of the grandparents
    const uint32_t nlist = counter(&v.st->gmerges);
    for (uint32_t li = blockIdx.x; li < nlist; li += gridDim.x) {
        const uint64_t u = v.upos[li];
        const uint32_t G = v.pn[lg + u];
        if (tid == 0) {
            // the first marked run under G merges it
            uint32_t first = 1;
            for (uint64_t e = u; e-- > 0 && v.pn[lg + e] == G;) {
                if (leaf_run_head(v, e) && v.f0[e] == 2u) {
                    first = 0;
                    break;
                }
            }
            s_first = first;
        }
        __syncthreads();
        const bool first = s_first != 0;
        __syncthreads();
        if (!first) continue;
        const uint32_t gc = v.pc[lg + u];
        // thread (p, l), tid < 256: leaf l of parent p, from the child lines
        uint32_t lref = kNone, lc = 0;
        if (tid < kSlots * kSlots) {
            const uint32_t p = static_cast<uint32_t>(tid) / kSlots, l = static_cast<uint32_t>(tid) % kSlots;
            if (p < gc) {
                const uint32_t P = t.ichild[static_cast<uint64_t>(G) * kSlots + p];
                if (l == 0) pid[p] = P;
                const uint32_t r = t.ichild[static_cast<uint64_t>(P) * kSlots + l];
                if (r != kNone) {
                    lref = r & ~kLeafTag;
                    const uint32_t c = t.lmeta[lref].x;
                    lc = c < kSlots ? c : kSlots;
                }
            }
        }
        uint32_t nleaf, T;
        const uint32_t lpos = block_excl_scan<uint32_t>(lref != kNone ? 1u : 0u, sh, &nleaf);
        const uint32_t kpos = block_excl_scan<uint32_t>(lc, sh, &T);
        if (lref != kNone) {
            lid[lpos] = lref;
            const uint64_t src = static_cast<uint64_t>(lref) * kSlots;
            for (uint32_t j = 0; j < lc; ++j) {
                mk[kpos + j] = t.lkeys[src + j];
                mv[kpos + j] = t.lvals[src + j];
            }
        }
        __syncthreads();
        if (tid == 0) s_next = nleaf ? t.lmeta[lid[nleaf - 1]].y : kNone;
        const bool root = h == 3;
        uint32_t n1, n0;
        const uint32_t w0 = (T + kSlots - 1) / kSlots, w1 = (T + kSlots * kSlots - 1) / (kSlots * kSlots);
        if (root && T <= kSlots) {
            n1 = 0;
            n0 = 1;
        } else if (root && T <= kSlots * kSlots) {
            n1 = 1;
            n0 = w0 > 2u ? w0 : 2u;
        } else {
            n1 = w1 > (root ? 2u : kHalf) ? w1 : (root ? 2u : kHalf);
            n0 = w0 > kHalf * n1 ? w0 : kHalf * n1;
        }
        const bool fail = (!root && T < kHalf * kHalf * kHalf) || n1 > gc || n0 > nleaf;
        __syncthreads();
        if (fail) {
            if (tid == 0) atomicOr(&v.st->rebuild, 1u);
            __syncthreads();
            continue;
        }
        // leaves: leaf j (j < n0) takes pairs [j q0 + min(j, r0), + len)
        const uint32_t q0 = T / n0, r0 = T % n0;
        auto leaf_end = [&](uint32_t j) { return (j + 1) * q0 + (j + 1 < r0 ? j + 1 : r0); };
        if (static_cast<uint32_t>(tid) < nleaf) {
            const uint32_t j = static_cast<uint32_t>(tid);
            const uint64_t dst = static_cast<uint64_t>(lid[j]) * kSlots;
            if (j < n0) {
                const uint32_t start = j * q0 + (j < r0 ? j : r0), len = leaf_end(j) - start;
                for (uint32_t s2 = 0; s2 < kSlots; ++s2) {
                    t.lkeys[dst + s2] = s2 < len ? mk[start + s2] : (len ? mk[start + len - 1] : kmax<K>());
                    t.lvals[dst + s2] = s2 < len ? mv[start + s2] : kmax<K>();
                }
                t.lmeta[lid[j]] = make_uint2(len, j + 1 < n0 ? lid[j + 1] : s_next);
            } else {
                for (uint32_t s2 = 0; s2 < kSlots; ++s2) {
                    t.lkeys[dst + s2] = kmax<K>();
                    t.lvals[dst + s2] = kmax<K>();
                }
                t.lmeta[lid[j]] = make_uint2(0u, kNone);
            }
        }
        // parents: parent i (i < n1) takes leaves [i q1 + min(i, r1), + c)
        const uint32_t q1 = n1 ? n0 / n1 : 0, r1 = n1 ? n0 % n1 : 0;
        auto par_first = [&](uint32_t i) { return i * q1 + (i < r1 ? i : r1); };
        if (n1 && tid < kSlots * kSlots) {
            const uint32_t i = static_cast<uint32_t>(tid) / kSlots, s2 = static_cast<uint32_t>(tid) % kSlots;
            if (i < n1) {
                const uint32_t a = par_first(i), c = par_first(i + 1) - a;
                const uint64_t P = pid[i];
                t.ichild[P * kSlots + s2] = s2 < c ? (lid[a + s2] | kLeafTag) : kNone;
                t.ikeys[P * kSlots + s2] = s2 + 1 < c ? mk[leaf_end(a + s2) - 1] : kmax<K>();
            }
        }
        if (n1 >= 2 && tid < kSlots) {
            const uint32_t s2 = static_cast<uint32_t>(tid);
            t.ichild[static_cast<uint64_t>(G) * kSlots + s2] = s2 < n1 ? pid[s2] : kNone;
            t.ikeys[static_cast<uint64_t>(G) * kSlots + s2] =
                s2 + 1 < n1 ? mk[leaf_end(par_first(s2 + 1) - 1) - 1] : kmax<K>();
        }
        if (tid == 0) {
            note_inner_write(v, h - 3);  // G and its parents, or the root that replaces G
            if (root && n1 == 0) {
                t.hdr->root = lid[0] | kLeafTag;
                t.hdr->height = 1;
            } else if (root && n1 == 1) {
                t.hdr->root = pid[0];
                t.hdr->height = 2;
            } else if (!root) {
                const K top = mk[T - 1];
                for (int l = h - 4; l >= 0; --l) {
                    const uint64_t o2 = static_cast<uint64_t>(l) * v.Bm + u;
                    if (v.pi[o2] + 1u < v.pc[o2]) {
                        t.ikeys[static_cast<uint64_t>(v.pn[o2]) * kSlots + v.pi[o2]] = top;
                        note_inner_write(v, l);
                        break;
                    }
                }
            }
        }
        __syncthreads();
    }
}

template <class K>
__global__ __launch_bounds__(1024) void k_del_merge2(TreeView<K> t, Ins<K> v) {
    ph_del_merge2<K>(t, v);
}

// Commit the count and the epoch, then refresh the top-levels mirror if a
// mirrored node changed, else only its key count (one launch).
template <class K, int NT>
__device__ __forceinline__ void ph_del_commit(TreeView<K> t, Ins<K> v) {
    if (threadIdx.x == 0 && !(t.hdr->error & kErrInternal)) {
        const uint32_t d = counter(&v.st->deleted);
        if (d) {
            t.hdr->n_keys -= d;
            t.hdr->epoch += 1;
        }
    }
    __syncthreads();
    if (counter(&v.st->mirror_dirty)) {
        mirror_refresh_body<K, NT>(t);
    } else if (threadIdx.x == 0) {
        reinterpret_cast<MirrorHeader*>(t.mirror)->n_keys = t.hdr->n_keys;
    }
}

template <class K>
__global__ __launch_bounds__(256) void k_del_commit(TreeView<K> t, Ins<K> v, uint64_t* host_word, uint32_t seq) {
    ph_del_commit<K, 256>(t, v);
    // the call's number and the rebuild flag (raised by the merge kernels
    // before this one), in one word, straight into host memory
    if (host_word && threadIdx.x == 0) {
        const uint64_t w = (static_cast<uint64_t>(seq) << 32) | (counter(&v.st->rebuild) ? 1u : 0u);
        __hip_atomic_store(host_word, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// A batch of at most kDelFusedMax keys in one launch: the batch path's
// phases, one after the other in a single 1024-thread workgroup (a grid of
// one workgroup runs each phase's loops over one workgroup), so the tree it
// leaves is the batch path's.  The batch is ranked in LDS (by key, then by
// position, the order of the batch path's sort); the parent merges run one
// per wave, the grandparent merges one after the other on the whole
// workgroup.  The workgroup's waves share one CU and its L1, so a barrier
// with its workgroup-scope fences orders the phases' plain loads and stores;
// the counters raised with atomics are read past the L1 (counter()).  A
// device-scope fence here would write back and invalidate the L2 at every
// phase.
constexpr int kDelOneBlock = 1024;
constexpr uint32_t kDelFusedMax = 64;

__device__ __forceinline__ void phase_boundary() {
    __syncthreads();
}

template <class K>
__global__ __launch_bounds__(kDelOneBlock) void k_del_small(TreeView<K> t, Ins<K> v, const K* __restrict__ keys,
                                                            uint32_t B, uint8_t* __restrict__ status,
                                                            uint64_t* host_word, uint32_t seq) {
    __shared__ K s_rk[kDelFusedMax];
    __shared__ K s_sk[kDelFusedMax];
    __shared__ uint32_t s_si[kDelFusedMax];
    __shared__ uint32_t sh[33];
    __shared__ MergeLds<K> s_merge[kDelOneBlock / 64];
    const uint32_t tid = threadIdx.x;
    uint32_t* st = reinterpret_cast<uint32_t*>(v.st);
    for (uint32_t i = tid; i < sizeof(InsState) / 4; i += kDelOneBlock) st[i] = 0;
    if (tid < B) s_rk[tid] = keys[tid];
    phase_boundary();
    // each key's stable rank in the batch
    if (tid < B) {
        const K k0 = s_rk[tid];
        const uint32_t c = stable_rank(s_rk, B, k0, tid);
        s_sk[c] = k0;
        s_si[c] = tid;
    }
    phase_boundary();
    // the distinct keys; a repeat reports ABSENT (an earlier occurrence
    // deletes the key)
    const bool in = tid < B;
    const bool head = in && (tid == 0 || s_sk[tid] != s_sk[tid - 1]);
    if (in) {
        v.sk[tid] = s_sk[tid];
        v.si[tid] = s_si[tid];  // locate writes each distinct key's status through it
        if (!head) status[s_si[tid]] = 0;
    }
    uint32_t U;
    const uint32_t pos = block_excl_scan<uint32_t>(head ? 1u : 0u, sh, &U);
    if (head) {
        v.uk[pos] = s_sk[tid];
        v.upos[pos] = tid;
    }
    if (tid == 0) {
        v.st->U = U;
        v.st->height = t.hdr->height;
    }
    phase_boundary();
    ph_locate<K, 16, 1, 2, kDelOneBlock>(t, v, status);
    phase_boundary();
    ph_del_leaf<K>(t, v);
    phase_boundary();
    ph_del_list<K>(t, v);
    phase_boundary();
    ph_del_merge<K>(t, v, false, tid / 64, kDelOneBlock / 64, s_merge[tid / 64]);
    phase_boundary();
    ph_del_merge2<K>(t, v);
    phase_boundary();
    ph_del_commit<K, kDelOneBlock>(t, v);
    // the call's number and the rebuild flag, in one word, straight into
    // host memory (the merges that raise the flag are behind the barriers
    // above): the host waits for this word rather than for the stream
    if (host_word && tid == 0) {
        const uint64_t w = (static_cast<uint64_t>(seq) << 32) | (counter(&v.st->rebuild) ? 1u : 0u);
        __hip_atomic_store(host_word, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

static std::atomic<int> g_one_launch_delete{1};
int set_one_launch_delete(int on) { return g_one_launch_delete.exchange(on ? 1 : 0, std::memory_order_relaxed); }
static bool one_launch_delete_on() { return g_one_launch_delete.load(std::memory_order_relaxed) != 0; }

// Copy every pair of the leaves that hold keys (cleared leaves hold none).
template <class K>
__global__ void k_del_collect(TreeView<K> t, uint32_t leaves, K* __restrict__ ok, K* __restrict__ ov, uint64_t cap,
                              unsigned long long* __restrict__ n) {
    for (uint64_t l = gtid(); l < leaves; l += gstride()) {
        const uint32_t c = t.lmeta[l].x < kSlots ? t.lmeta[l].x : kSlots;
        if (c == 0) continue;
        const uint64_t at = atomicAdd(n, static_cast<unsigned long long>(c));
        if (at + c > cap) continue;  // more pairs than the tree counts: the host reports it
        for (uint32_t j = 0; j < c; ++j) {
            ok[at + j] = t.lkeys[l * kSlots + j];
            ov[at + j] = t.lvals[l * kSlots + j];
        }
    }
}

template <class K>
const uint32_t* launch_delete(const TreeView<K>& t, const InsertCtx& c, const K* keys, uint64_t B, uint8_t* status,
                              uint64_t* host_word, uint32_t seq, bool* flag_on_host, hipStream_t s) {
    *flag_on_host = false;
    Ins<K> v;
    carve<K>(&v, c.scratch, c.max_batch, c.leaf_cap, c.inner_cap);
    const uint32_t gB = grid_for(B, kBlk);
    if (B <= kDelFusedMax && one_launch_delete_on()) {
        const uint32_t lds = MirrorLayout<K>::bytes(mirror_nodes_for_levels(2));
        hipLaunchKernelGGL(k_del_small<K>, dim3(1), dim3(kDelOneBlock), lds, s, t, v, keys,
                           static_cast<uint32_t>(B), status, host_word, seq);
        *flag_on_host = host_word != nullptr;
        return &v.st->rebuild;
    }
    if (B <= kSmallInsert) {
        rank_sort_small<K>(keys, static_cast<uint32_t>(B), v.sk, v.si, reinterpret_cast<uint32_t*>(v.st),
                           static_cast<uint32_t>(sizeof(InsState) / 4), s);
        hipLaunchKernelGGL(k_del_small_prefix<K>, dim3(1), dim3(1024), 0, s, v, t.hdr, static_cast<uint32_t>(B),
                           status);
    } else {
        hipLaunchKernelGGL(k_init<K>, dim3(1), dim3(kBlk), 0, s, v, t.hdr);
        sort_from<K>(keys, v.sk, v.si, v.sk2, v.si2, B, v.sort_tmp, s, &t.hdr->error, kErrInternal);
        hipLaunchKernelGGL(k_del_heads<K>, dim3(gB), dim3(kBlk), 0, s, v, B, status);
        scan_exclusive<uint32_t>(v.f0, v.f1, &v.st->U, nullptr, B, v.scan_tmp, s);
        hipLaunchKernelGGL(k_del_unique<K>, dim3(gB), dim3(kBlk), 0, s, v, B);
    }
    launch_locate<K>(t, v, c.cfg, B, status, s);
    const uint64_t gl = grid_for(B * kSlots, kBlk);
    hipLaunchKernelGGL(k_del_leaf<K>, dim3(gl < 65536 ? static_cast<uint32_t>(gl) : 65536u), dim3(kBlk), 0, s, t, v);
    const bool ordered = B > kDelListScan;
    if (ordered) {
        scan_exclusive<uint32_t>(v.nu, v.nleaf, &v.st->merges, &v.st->U, B, v.scan_tmp, s);
        hipLaunchKernelGGL(k_del_list_ordered<K>, dim3(gB), dim3(kBlk), 0, s, t, v);
    } else {
        hipLaunchKernelGGL(k_del_list<K>, dim3(gB), dim3(kBlk), 0, s, t, v);
    }
    const uint32_t gm = B < 16384 ? static_cast<uint32_t>(B) : 16384u;
    hipLaunchKernelGGL(k_del_merge<K>, dim3(gm), dim3(64), 0, s, t, v, ordered);
    hipLaunchKernelGGL(k_del_merge2<K>, dim3(B < 256 ? static_cast<uint32_t>(B) : 256u), dim3(1024), 0, s, t, v);
    hipLaunchKernelGGL(k_del_commit<K>, dim3(1), dim3(256), 0, s, t, v, host_word, seq);
    *flag_on_host = host_word != nullptr;
    return &v.st->rebuild;
}

template <class K>
void launch_delete_collect(const TreeView<K>& t, uint32_t leaves, K* ok, K* ov, uint64_t cap,
                           unsigned long long* n, hipStream_t s) {
    const uint32_t g = grid_for(leaves ? leaves : 1, kBlk);
    hipLaunchKernelGGL(k_del_collect<K>, dim3(g < 4096 ? g : 4096), dim3(kBlk), 0, s, t, leaves, ok, ov, cap, n);
}

template const uint32_t* launch_delete<uint32_t>(const TreeView<uint32_t>&, const InsertCtx&, const uint32_t*,
                                                 uint64_t, uint8_t*, uint64_t*, uint32_t, bool*, hipStream_t);
template const uint32_t* launch_delete<uint64_t>(const TreeView<uint64_t>&, const InsertCtx&, const uint64_t*,
                                                 uint64_t, uint8_t*, uint64_t*, uint32_t, bool*, hipStream_t);
template void launch_delete_collect<uint32_t>(const TreeView<uint32_t>&, uint32_t, uint32_t*, uint32_t*, uint64_t,
                                              unsigned long long*, hipStream_t);
template void launch_delete_collect<uint64_t>(const TreeView<uint64_t>&, uint32_t, uint64_t*, uint64_t*, uint64_t,
                                              unsigned long long*, hipStream_t);

}  // namespace gt
