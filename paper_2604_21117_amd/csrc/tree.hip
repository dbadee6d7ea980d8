// Host runtime of the tree library and its C ABI (gtree.h).
//
// A gt_tree handle records where the tree lives in the caller's arena and
// which launch configuration the search kernels use.  Every entry point
// checks its arguments on the host, then enqueues kernels on the caller's
// stream without synchronising (tree_build, tree_stats, tree_export and
// tree_device_error are the documented exceptions).
#include <chrono>
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <cstddef>
#include <vector>
#include <algorithm>

#include "../../include/gtree.h"
#include "../../include/gtree_testing.h"
#include "common.h"
#include "kernels.h"
#include "prims.h"
#include "insert.h"
#include "handle.h"

using namespace gt;

namespace {

constexpr uint64_t kAlign = 256;
uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool params_ok(const gt_params* p) {
    if (!p) return false;
    if (p->key_bytes != 4 && p->key_bytes != 8) return false;
    if (p->fanout != 0 && p->fanout != 16) return false;
    if (p->leaf_cap != 0 && p->leaf_cap != 16) return false;
    if (p->fill != 0.0f && (p->fill < 0.5f || p->fill > 1.0f)) return false;
    if (p->lanes_per_query != 0 && p->lanes_per_query != 4 && p->lanes_per_query != 8 && p->lanes_per_query != 16)
        return false;
    if (p->lds_levels > 4) return false;
    if (p->queries_per_group != 0 && p->queries_per_group != 1 && p->queries_per_group != 2 &&
        p->queries_per_group != 4)
        return false;
    if (p->sorted_mode != 0) return false;
    if (p->value_coload > 2 || p->xcd_split > 2 || p->leaf_stream > 2 || p->reserved != 0) return false;
    return true;
}

float fill_of(const gt_params* p) { return p->fill == 0.0f ? 1.0f : p->fill; }
uint64_t max_batch_of(const gt_params* p) { return p->max_batch ? p->max_batch : (1ull << 20); }

uint64_t leaf_rec_bytes(int kb) { return 2ull * kSlots * kb + 8; }
uint64_t inner_rec_bytes(int kb) { return static_cast<uint64_t>(kSlots) * (kb + 4); }

uint64_t mirror_bytes(int kb) {
    return align_up(kb == 8 ? MirrorLayout<uint64_t>::global_bytes() : MirrorLayout<uint32_t>::global_bytes());
}

// nodes a level of `items` entries packs into (cap per node after fill, at
// least cap/2 per node when there are two or more)
uint64_t pack_count(uint64_t items, uint64_t cap, double fill) {
    uint64_t per = static_cast<uint64_t>(cap * fill);
    if (per < 1) per = 1;
    uint64_t a = (items + per - 1) / per;
    uint64_t b = items / ((cap + 1) / 2);
    uint64_t c = a < b ? a : b;
    return c < 1 ? 1 : c;
}

std::vector<uint64_t> level_sizes_for(uint64_t n, double fill) {
    std::vector<uint64_t> v;
    uint64_t L = pack_count(n, kSlots, fill);
    v.push_back(L);
    uint64_t c = L;
    while (c > 1) {
        c = pack_count(c, kSlots, fill);
        v.push_back(c);
    }
    return v;
}

// inner nodes needed for `leaves` leaves when every non-root inner node has
// at least 8 children
uint64_t inner_cap_for(uint64_t leaves) { return leaves / 7 + 2 * kMaxLevels; }

// Largest height a tree with at most `leaf_cap` leaves can have: a non-root
// inner node has at least 8 children and an inner root at least 2, so a tree
// of height h >= 2 has at least 2 * 8^(h-2) leaves.
uint32_t height_cap(uint64_t leaf_cap) {
    uint32_t h = 1;
    uint64_t need = 2;  // leaves a tree of height h + 1 needs at least
    while (need <= leaf_cap && h < static_cast<uint32_t>(kMaxLevels)) {
        ++h;
        need *= 8;
    }
    return h;
}

uint64_t fixed_bytes(int kb, uint64_t max_batch, uint64_t leaf_cap) {
    return align_up(sizeof(DevHeader)) + mirror_bytes(kb) +
           align_up(insert_scratch_bytes(max_batch, kb, leaf_cap, inner_cap_for(leaf_cap)));
}

void layout(gt_tree* t, uint8_t* arena, uint64_t leaf_cap) {
    const int kb = t->kb;
    uint64_t off = 0;
    t->arena = arena;
    t->hdr = reinterpret_cast<DevHeader*>(arena + off);
    off += align_up(sizeof(DevHeader));
    t->mirror = arena + off;
    off += mirror_bytes(kb);
    t->scratch = arena + off;
    t->scratch_bytes = align_up(insert_scratch_bytes(t->max_batch, kb, leaf_cap, inner_cap_for(leaf_cap)));
    off += t->scratch_bytes;
    t->leaf_cap = leaf_cap;
    t->inner_cap = inner_cap_for(leaf_cap);
    t->ikeys = arena + off;
    off += align_up(t->inner_cap * kSlots * kb);
    t->ichild = reinterpret_cast<uint32_t*>(arena + off);
    off += align_up(t->inner_cap * kSlots * 4);
    t->lkeys = arena + off;
    off += align_up(leaf_cap * kSlots * kb);
    t->lvals = arena + off;
    off += align_up(leaf_cap * kSlots * kb);
    t->lmeta = reinterpret_cast<uint2*>(arena + off);
    off += align_up(leaf_cap * 8);
    t->arena_bytes = off;
}

uint64_t bytes_for_leaf_cap(int kb, uint64_t max_batch, uint64_t leaf_cap) {
    uint64_t ic = inner_cap_for(leaf_cap);
    return fixed_bytes(kb, max_batch, leaf_cap) + align_up(ic * kSlots * kb) + align_up(ic * kSlots * 4) +
           2 * align_up(leaf_cap * kSlots * kb) + align_up(leaf_cap * 8);
}

#define HIP_TRY(x)                                  \
    do {                                            \
        if ((x) != hipSuccess) return GT_ERR_HIP;   \
    } while (0)

template <class K>
gt_status build_t(gt_tree* t, const void* keys, const void* values, uint64_t n, hipStream_t s) {
    const double fill = fill_of(&t->p);
    std::vector<uint64_t> sizes = level_sizes_for(n, fill);
    if (sizes.size() > static_cast<size_t>(kMaxLevels)) return GT_ERR_CAPACITY;
    if (sizes[0] > t->leaf_cap) return GT_ERR_CAPACITY;
    uint64_t inner_total = 0;
    for (size_t i = 1; i < sizes.size(); ++i) inner_total += sizes[i];
    if (inner_total > t->inner_cap) return GT_ERR_CAPACITY;
    if (t->leaf_cap >= kLeafTag || t->inner_cap >= kLeafTag) return GT_ERR_CAPACITY;

    // temporary buffers: sorted keys/idx + ping-pong, sorted values, sort
    // scratch, per-level maxima, duplicate flag
    const uint64_t nn = n ? n : 1;
    uint64_t maxsz = 0;
    for (uint64_t v : sizes) maxsz = std::max(maxsz, v);
    const uint64_t b_keys = align_up(nn * sizeof(K)), b_idx = align_up(nn * 4);
    const uint64_t b_sort = align_up(sort_tmp_bytes(nn, sizeof(K)));
    const uint64_t b_max = align_up(2 * maxsz * sizeof(K));
    const uint64_t total = 3 * b_keys + 2 * b_idx + b_sort + b_max + kAlign;
    uint8_t* tmp = nullptr;
    HIP_TRY(hipMalloc(&tmp, total));
    uint8_t* p = tmp;
    K* sk = reinterpret_cast<K*>(p); p += b_keys;
    K* sk2 = reinterpret_cast<K*>(p); p += b_keys;
    K* sv = reinterpret_cast<K*>(p); p += b_keys;
    uint32_t* si = reinterpret_cast<uint32_t*>(p); p += b_idx;
    uint32_t* si2 = reinterpret_cast<uint32_t*>(p); p += b_idx;
    void* stmp = p; p += b_sort;
    K* maxbuf = reinterpret_cast<K*>(p); p += b_max;
    uint32_t* dflag = reinterpret_cast<uint32_t*>(p);

    gt_status st = GT_OK;
    uint32_t hflag = 0;
    do {
        if (hipMemsetAsync(dflag, 0, 4, s) != hipSuccess) { st = GT_ERR_HIP; break; }
        if (n) {
            // (key, position) pairs sorted by key; positions come from the sort
            sort_from<K>(reinterpret_cast<const K*>(keys), sk, si, sk2, si2, n, stmp, s, dflag, 2u);  // bit 0: duplicates (below)
            launch_gather<K>(reinterpret_cast<const K*>(values), si, sv, n, s);
            launch_dup_check<K>(sk, n, dflag, s);
        }
        if (hipMemcpyAsync(&hflag, dflag, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            st = GT_ERR_HIP;
            break;
        }
        if (hflag & 2u) { st = GT_ERR_DEVICE; break; }  // the sort gave up
        if (hflag) { st = GT_ERR_DUPLICATE; break; }
        TreeView<K> v = view<K>(t);
        launch_build<K>(v, sk, sv, n, sizes.data(), static_cast<int>(sizes.size()), maxbuf, s);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) st = GT_ERR_HIP;
        t->h_bound = static_cast<uint32_t>(sizes.size());
    } while (0);
    hipStreamSynchronize(s);
    hipFree(tmp);
    return st;
}

// After a delete batch whose merges could not keep a leaf parent at least
// half full: rebuild the tree in place from the pairs its leaves hold (the
// bulk load fixes every level and the height), keeping the error word and
// moving the epoch on.
template <class K>
gt_status delete_rebuild_t(gt_tree* t, hipStream_t s) {
    DevHeader h;
    HIP_TRY(hipMemcpyAsync(&h, t->hdr, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const uint64_t n = h.n_keys;
    uint8_t* buf = nullptr;
    const uint64_t b_keys = align_up((n ? n : 1) * sizeof(K));
    HIP_TRY(hipMalloc(&buf, 2 * b_keys + kAlign));
    K* ok = reinterpret_cast<K*>(buf);
    K* ov = reinterpret_cast<K*>(buf + b_keys);
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(buf + 2 * b_keys);
    gt_status st = GT_OK;
    unsigned long long got = 0;
    do {
        if (hipMemsetAsync(cnt, 0, sizeof *cnt, s) != hipSuccess) { st = GT_ERR_HIP; break; }
        launch_delete_collect<K>(view<K>(t), h.leaf_used, ok, ov, n, cnt, s);
        if (hipMemcpyAsync(&got, cnt, sizeof got, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            st = GT_ERR_HIP;
            break;
        }
        if (got != n) { st = GT_ERR_DEVICE; break; }
        st = build_t<K>(t, ok, ov, n, s);
        if (st != GT_OK) break;
        const uint32_t keep[2] = {h.error, h.epoch + 1};  // DevHeader: error, then epoch
        static_assert(offsetof(DevHeader, epoch) == offsetof(DevHeader, error) + 4, "header layout");
        if (hipMemcpyAsync(&t->hdr->error, keep, sizeof keep, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            st = GT_ERR_HIP;
    } while (0);
    hipStreamSynchronize(s);
    hipFree(buf);
    return st;
}

}  // namespace

namespace {

// Copy what training a learned index reads -- the header, the child
// references of the inner nodes in use and the keys and {count, next} of
// the leaves in use -- from one arena layout to another.  The counts in use
// come from the source header, so the copy follows the tree the stream
// order leaves it.  16-byte words, grid-stride.
__global__ void k_train_copy(const DevHeader* __restrict__ sh, DevHeader* __restrict__ dh,
                             const uint4* __restrict__ sic, uint4* __restrict__ dic,
                             const uint4* __restrict__ slk, uint4* __restrict__ dlk,
                             const uint4* __restrict__ slm, uint4* __restrict__ dlm, uint32_t key_bytes) {
    const uint64_t ni = sh->inner_used, nl = sh->leaf_used;
    const uint64_t n_ic = ni * kSlots * 4 / 16, n_lk = nl * kSlots * key_bytes / 16, n_lm = (nl * 8 + 15) / 16;
    const uint64_t tid = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    if (tid == 0) *dh = *sh;
    for (uint64_t i = tid; i < n_ic; i += stride) dic[i] = sic[i];
    for (uint64_t i = tid; i < n_lk; i += stride) dlk[i] = slk[i];
    for (uint64_t i = tid; i < n_lm; i += stride) dlm[i] = slm[i];
}

}  // namespace

gt_status gt_tree_copy_for_training(const gt_tree* t, gt_tree* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_train_copy, dim3(2048), dim3(256), 0, s, t->hdr, dst->hdr,
                       reinterpret_cast<const uint4*>(t->ichild), reinterpret_cast<uint4*>(dst->ichild),
                       reinterpret_cast<const uint4*>(t->lkeys), reinterpret_cast<uint4*>(dst->lkeys),
                       reinterpret_cast<const uint4*>(t->lmeta), reinterpret_cast<uint4*>(dst->lmeta),
                       static_cast<uint32_t>(t->kb));
    return hipGetLastError() == hipSuccess ? GT_OK : GT_ERR_HIP;
}

gt_tree* gt_tree_clone_handle(const gt_tree* t, uint8_t* arena) {
    gt_tree* c = new gt_tree(*t);
    c->h_flag = nullptr;
    c->d_flag = nullptr;
    c->wide = nullptr;
    c->inserts = 0;
    c->deletes = 0;
    layout(c, arena, t->leaf_cap);
    return c;
}

extern "C" {

const char* gt_status_str(gt_status s) {
    switch (s) {
        case GT_OK: return "ok";
        case GT_ERR_INVALID: return "invalid argument";
        case GT_ERR_DUPLICATE: return "duplicate key";
        case GT_ERR_CAPACITY: return "capacity exceeded";
        case GT_ERR_ADMISSION: return "admission refused";
        case GT_ERR_HIP: return "HIP runtime error";
        case GT_ERR_DEVICE: return "device error";
    }
    return "unknown status";
}

uint32_t gt_set_sort_spin_limit(uint32_t limit) { return set_sort_spin_limit(limit); }
int gt_set_single_key_insert(int enable) { return set_single_key_insert(enable); }
int gt_set_one_launch_insert(int enable) { return set_one_launch_insert(enable); }
int gt_set_one_launch_delete(int enable) { return set_one_launch_delete(enable); }

uint64_t tree_arena_bytes(const gt_params* p, uint64_t n, uint64_t leaf_slack) {
    if (wide_selected(p)) return wide_arena_bytes(p, n);  // static: no headroom
    if (!params_ok(p)) return 0;
    std::vector<uint64_t> sizes = level_sizes_for(n, fill_of(p));
    return bytes_for_leaf_cap(static_cast<int>(p->key_bytes), max_batch_of(p), sizes[0] + leaf_slack);
}

gt_status tree_build(const gt_params* p, const void* keys, const void* values, uint64_t n, void* arena,
                     uint64_t arena_bytes, hipStream_t stream, gt_tree** out) {
    if (wide_selected(p)) {
        if (!out) return GT_ERR_INVALID;
        WideTree* w = nullptr;
        const gt_status st = wide_build(p, keys, values, n, arena, arena_bytes, stream, &w);
        if (st != GT_OK) return st;
        gt_tree* t = new gt_tree();
        t->p = *p;
        t->kb = static_cast<int>(p->key_bytes);
        t->arena = reinterpret_cast<uint8_t*>(arena);
        t->arena_bytes = w->arena_bytes;
        t->h_bound = w->height;
        t->wide = w;
        *out = t;
        return GT_OK;
    }
    if (!params_ok(p) || !arena || !out || (n && (!keys || !values))) return GT_ERR_INVALID;
    if (n >= (1ull << 36)) return GT_ERR_INVALID;
    const int kb = static_cast<int>(p->key_bytes);
    const uint64_t mb = max_batch_of(p);
    if (mb >= (1ull << 31)) return GT_ERR_INVALID;
    if (bytes_for_leaf_cap(kb, mb, 1) > arena_bytes) return GT_ERR_CAPACITY;
    // largest leaf capacity that fits the arena
    uint64_t lo = 1, hi = arena_bytes / leaf_rec_bytes(kb) + 1;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo + 1) / 2;
        if (bytes_for_leaf_cap(kb, mb, mid) <= arena_bytes) lo = mid; else hi = mid - 1;
    }
    if (lo >= kLeafTag - 1) lo = kLeafTag - 2;
    gt_tree* t = new gt_tree();
    t->p = *p;
    t->kb = kb;
    t->max_batch = mb;
    t->cfg.lanes = p->lanes_per_query ? static_cast<int>(p->lanes_per_query) : 8;
    t->cfg.queries_per_group = p->queries_per_group ? static_cast<int>(p->queries_per_group) : 2;
    t->cfg.lds_levels = p->lds_levels == 0 ? 2 : (p->lds_levels == 4 ? 0 : static_cast<int>(p->lds_levels));
    t->cfg.value_coload = p->value_coload == 2 ? 0 : 1;
    t->cfg.xcd_split = p->xcd_split == 1 ? 1 : 0;
    t->cfg.leaf_stream = static_cast<int>(p->leaf_stream);  // 0 by batch size, 1 both lines, 2 none
    // an explicit queries_per_group applies to every batch size
    t->cfg.large_qpg = p->queries_per_group ? 0 : 2;
    // lookup shape fields the caller left at 0 follow the batch size
    t->cfg.shape_auto = (p->lanes_per_query ? 0 : 1) | (p->queries_per_group ? 0 : 2) | (p->lds_levels ? 0 : 4);
    layout(t, reinterpret_cast<uint8_t*>(arena), lo);
    gt_status st = kb == 8 ? build_t<uint64_t>(t, keys, values, n, stream)
                           : build_t<uint32_t>(t, keys, values, n, stream);
    if (st != GT_OK) {
        delete t;
        return st;
    }
    *out = t;
    return GT_OK;
}

gt_status tree_lookup_batch(gt_tree* t, const void* keys, uint64_t B, void* values_out, uint8_t* found_out,
                            hipStream_t stream) {
    if (!t) return GT_ERR_INVALID;
    if (B == 0) return GT_OK;
    if (!keys || !values_out || !found_out) return GT_ERR_INVALID;
    if (t->wide) return wide_lookup(t->wide, keys, B, values_out, found_out, stream);
    if (t->kb == 8)
        launch_lookup<uint64_t>(view<uint64_t>(t), t->cfg, reinterpret_cast<const uint64_t*>(keys), B,
                                reinterpret_cast<uint64_t*>(values_out), found_out, stream);
    else
        launch_lookup<uint32_t>(view<uint32_t>(t), t->cfg, reinterpret_cast<const uint32_t*>(keys), B,
                                reinterpret_cast<uint32_t*>(values_out), found_out, stream);
    return hipGetLastError() == hipSuccess ? GT_OK : GT_ERR_HIP;
}

uint64_t tree_lookup_levelwise_workspace_bytes(const gt_tree* t, uint64_t B, uint32_t flags) {
    if (!t || t->wide || (flags & ~GT_LW_PRESORTED) != 0) return 0;
    return lw_layout(B, t->kb, (flags & GT_LW_PRESORTED) != 0).total;
}

gt_status tree_lookup_levelwise(gt_tree* t, const void* keys, uint64_t B, uint32_t flags, void* values_out,
                                uint8_t* found_out, void* workspace, uint64_t workspace_bytes, hipStream_t stream) {
    if (!t || t->wide) return GT_ERR_INVALID;
    if ((flags & ~GT_LW_PRESORTED) != 0) return GT_ERR_INVALID;
    if (B == 0) return GT_OK;
    if (!keys || !values_out || !found_out || !workspace) return GT_ERR_INVALID;
    if (B >= (1ull << 31)) return GT_ERR_INVALID;
    const bool presorted = (flags & GT_LW_PRESORTED) != 0;
    if (workspace_bytes < lw_layout(B, t->kb, presorted).total) return GT_ERR_CAPACITY;
    if (t->kb == 8)
        launch_lookup_levelwise<uint64_t>(view<uint64_t>(t), reinterpret_cast<const uint64_t*>(keys), B,
                                          presorted, t->h_bound, reinterpret_cast<uint64_t*>(values_out),
                                          found_out, workspace, stream);
    else
        launch_lookup_levelwise<uint32_t>(view<uint32_t>(t), reinterpret_cast<const uint32_t*>(keys), B,
                                          presorted, t->h_bound, reinterpret_cast<uint32_t*>(values_out),
                                          found_out, workspace, stream);
    return hipGetLastError() == hipSuccess ? GT_OK : GT_ERR_HIP;
}

gt_status tree_lookup_levelwise_noalloc(gt_tree* t, const void* keys, uint64_t B, uint32_t flags,
                                        void* values_out, uint8_t* found_out, hipStream_t stream) {
    if (!t || t->wide) return GT_ERR_INVALID;
    if ((flags & ~GT_LW_PRESORTED) != 0) return GT_ERR_INVALID;
    if (B == 0) return GT_OK;
    if (!keys || !values_out || !found_out) return GT_ERR_INVALID;
    if (B >= (1ull << 31)) return GT_ERR_INVALID;
    const bool presorted = (flags & GT_LW_PRESORTED) != 0;
    if (lw_layout(B, t->kb, presorted).total > kLwScratchBytes) return GT_ERR_CAPACITY;
    void* ws = nullptr;
    if (lw_scratch(&ws) != hipSuccess) return GT_ERR_HIP;
    if (t->kb == 8)
        launch_lookup_levelwise<uint64_t>(view<uint64_t>(t), reinterpret_cast<const uint64_t*>(keys), B,
                                          presorted, t->h_bound, reinterpret_cast<uint64_t*>(values_out),
                                          found_out, ws, stream);
    else
        launch_lookup_levelwise<uint32_t>(view<uint32_t>(t), reinterpret_cast<const uint32_t*>(keys), B,
                                          presorted, t->h_bound, reinterpret_cast<uint32_t*>(values_out),
                                          found_out, ws, stream);
    return hipGetLastError() == hipSuccess ? GT_OK : GT_ERR_HIP;
}

gt_status tree_delete_batch(gt_tree* t, const void* keys, uint64_t B, uint8_t* status_out, hipStream_t stream) {
    if (!t || t->wide) return GT_ERR_INVALID;
    if (B == 0) return GT_OK;
    if (!keys || !status_out) return GT_ERR_INVALID;
    if (B > t->max_batch) return GT_ERR_CAPACITY;
    InsertCtx c;
    c.scratch = t->scratch;
    c.scratch_bytes = t->scratch_bytes;
    c.max_batch = t->max_batch;
    c.inner_cap = t->inner_cap;
    c.leaf_cap = t->leaf_cap;
    c.cfg = t->cfg;
    // pinned, so that the flag goes straight to host memory (the first call
    // allocates it); the batch's last kernel stores it there itself
    if (!t->h_flag) {
        HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&t->h_flag), 64, hipHostMallocDefault));
        *t->h_flag = 0;  // no call has answered yet (call numbers start at 1)
        if (hipHostGetDevicePointer(reinterpret_cast<void**>(&t->d_flag), t->h_flag, 0) != hipSuccess)
            t->d_flag = nullptr;
    }
    bool on_host = false;
    const uint32_t seq = static_cast<uint32_t>(t->deletes + 1);
    const uint32_t* flag =
        t->kb == 8 ? launch_delete<uint64_t>(view<uint64_t>(t), c, reinterpret_cast<const uint64_t*>(keys), B,
                                             status_out, t->d_flag, seq, &on_host, stream)
                   : launch_delete<uint32_t>(view<uint32_t>(t), c, reinterpret_cast<const uint32_t*>(keys), B,
                                             status_out, t->d_flag, seq, &on_host, stream);
    HIP_TRY(hipGetLastError());
    t->deletes++;
    bool rebuild;
    if (on_host) {
        // the kernel stores (seq << 32 | flag) into the pinned word as its
        // answer: wait for that word, not for the stream (the stream's end
        // is checked now and then, so that a kernel that never stores it
        // cannot hold the call)
        // (the stream is asked at most every 50 us: a query takes the
        // runtime's locks and costs more than the wait it checks)
        const volatile uint64_t* w = t->h_flag;
        uint64_t got = 0;
        auto next = std::chrono::steady_clock::now() + std::chrono::microseconds(50);
        for (uint32_t i = 1;; ++i) {
            got = __atomic_load_n(w, __ATOMIC_ACQUIRE);
            if (static_cast<uint32_t>(got >> 32) == seq) break;
            __builtin_ia32_pause();
            if (i % 64 != 0) continue;
            const auto now = std::chrono::steady_clock::now();
            if (now < next) continue;
            next = now + std::chrono::microseconds(50);
            const hipError_t q = hipStreamQuery(stream);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) return GT_ERR_HIP;
            got = __atomic_load_n(w, __ATOMIC_ACQUIRE);
            if (static_cast<uint32_t>(got >> 32) != seq) return GT_ERR_HIP;
            break;
        }
        rebuild = (got & 0xffffffffu) != 0;
    } else {
        HIP_TRY(hipMemcpyAsync(t->h_flag, flag, 4, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        rebuild = (*t->h_flag & 0xffffffffu) != 0;
    }
    if (!rebuild) return GT_OK;
    return t->kb == 8 ? delete_rebuild_t<uint64_t>(t, stream) : delete_rebuild_t<uint32_t>(t, stream);
}

gt_status tree_range_batch(gt_tree* t, const void* lo, const void* hi, const uint32_t* max_out,
                           const uint64_t* out_offsets, uint64_t B, void* out_keys, void* out_values,
                           uint32_t* count_out, hipStream_t stream) {
    if (!t) return GT_ERR_INVALID;
    if (B == 0) return GT_OK;
    if (!lo || !hi || !max_out || !out_offsets || !out_keys || !out_values || !count_out) return GT_ERR_INVALID;
    if (t->wide)
        return wide_range(t->wide, lo, hi, max_out, out_offsets, B, out_keys, out_values, count_out, stream);
    if (t->kb == 8)
        launch_range<uint64_t>(view<uint64_t>(t), t->cfg, reinterpret_cast<const uint64_t*>(lo),
                               reinterpret_cast<const uint64_t*>(hi), max_out, out_offsets, B,
                               reinterpret_cast<uint64_t*>(out_keys), reinterpret_cast<uint64_t*>(out_values),
                               count_out, stream);
    else
        launch_range<uint32_t>(view<uint32_t>(t), t->cfg, reinterpret_cast<const uint32_t*>(lo),
                               reinterpret_cast<const uint32_t*>(hi), max_out, out_offsets, B,
                               reinterpret_cast<uint32_t*>(out_keys), reinterpret_cast<uint32_t*>(out_values),
                               count_out, stream);
    return hipGetLastError() == hipSuccess ? GT_OK : GT_ERR_HIP;
}

gt_status tree_insert_batch(gt_tree* t, const void* keys, const void* values, uint64_t B, uint8_t* status_out,
                            hipStream_t stream) {
    if (!t || t->wide) return GT_ERR_INVALID;
    if (B == 0) return GT_OK;
    if (!keys || !values || !status_out) return GT_ERR_INVALID;
    if (B > t->max_batch) return GT_ERR_CAPACITY;
    InsertCtx c;
    c.scratch = t->scratch;
    c.scratch_bytes = t->scratch_bytes;
    c.max_batch = t->max_batch;
    c.inner_cap = t->inner_cap;
    c.leaf_cap = t->leaf_cap;
    c.cfg = t->cfg;
    if (t->kb == 8)
        launch_insert<uint64_t>(view<uint64_t>(t), c, reinterpret_cast<const uint64_t*>(keys),
                                reinterpret_cast<const uint64_t*>(values), B, status_out, stream);
    else
        launch_insert<uint32_t>(view<uint32_t>(t), c, reinterpret_cast<const uint32_t*>(keys),
                                reinterpret_cast<const uint32_t*>(values), B, status_out, stream);
    // the batch may grow the tree on the device; the host keeps a bound
    const uint32_t hc = height_cap(t->leaf_cap);
    if (hc > t->h_bound) t->h_bound = hc;
    t->inserts++;
    return hipGetLastError() == hipSuccess ? GT_OK : GT_ERR_HIP;
}

gt_status tree_destroy(gt_tree* t) {
    if (!t) return GT_ERR_INVALID;
    if (t->h_flag) hipHostFree(t->h_flag);
    delete t->wide;
    delete t;
    return GT_OK;
}

gt_status tree_stats(gt_tree* t, gt_tree_stats* out, hipStream_t stream) {
    if (!t || !out) return GT_ERR_INVALID;
    if (t->wide) return wide_stats(t->wide, out, stream);
    DevHeader h;
    HIP_TRY(hipMemcpyAsync(&h, t->hdr, sizeof h, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    memset(out, 0, sizeof *out);
    out->n_keys = h.n_keys;
    out->height = h.height;
    out->root = h.root;
    out->inner_used = h.inner_used;
    out->inner_cap = t->inner_cap;
    out->leaf_used = h.leaf_used;
    out->leaf_cap = t->leaf_cap;
    out->arena_bytes = t->arena_bytes;
    out->max_batch = t->max_batch;
    out->error_word = h.error;
    out->key_bytes = static_cast<uint32_t>(t->kb);
    return GT_OK;
}

gt_status tree_device_error(gt_tree* t, hipStream_t stream) {
    if (!t) return GT_ERR_INVALID;
    if (t->wide) return wide_device_error(t->wide, stream);
    uint32_t e = 0;
    HIP_TRY(hipMemcpyAsync(&e, &t->hdr->error, 4, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (e) {
        HIP_TRY(hipMemsetAsync(&t->hdr->error, 0, 4, stream));
        HIP_TRY(hipStreamSynchronize(stream));
    }
    if (e & kErrInternal) return GT_ERR_DEVICE;
    if (e & kErrCapacity) return GT_ERR_CAPACITY;
    return GT_OK;
}

gt_status tree_export(gt_tree* t, void* host_buf, uint64_t* bytes, hipStream_t stream) {
    if (!t || !bytes) return GT_ERR_INVALID;
    if (t->wide) return wide_export(t->wide, host_buf, bytes, stream);
    DevHeader h;
    HIP_TRY(hipMemcpyAsync(&h, t->hdr, sizeof h, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    const int kb = t->kb;
    const uint64_t ni = h.inner_used, nl = h.leaf_used;
    const uint64_t need = 48 + ni * inner_rec_bytes(kb) + nl * leaf_rec_bytes(kb);
    if (!host_buf) {
        *bytes = need;
        return GT_OK;
    }
    if (*bytes < need) return GT_ERR_CAPACITY;
    std::vector<uint8_t> ik(ni * kSlots * kb), ic(ni * kSlots * 4), lk(nl * kSlots * kb), lv(nl * kSlots * kb),
        lm(nl * 8);
    if (ni) {
        HIP_TRY(hipMemcpyAsync(ik.data(), t->ikeys, ik.size(), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipMemcpyAsync(ic.data(), t->ichild, ic.size(), hipMemcpyDeviceToHost, stream));
    }
    if (nl) {
        HIP_TRY(hipMemcpyAsync(lk.data(), t->lkeys, lk.size(), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipMemcpyAsync(lv.data(), t->lvals, lv.size(), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipMemcpyAsync(lm.data(), t->lmeta, lm.size(), hipMemcpyDeviceToHost, stream));
    }
    HIP_TRY(hipStreamSynchronize(stream));
    uint8_t* o = reinterpret_cast<uint8_t*>(host_buf);
    uint32_t hdr[10] = {0x58455447u, static_cast<uint32_t>(kb), kSlots, kSlots, h.height, h.root,
                        h.first_leaf, static_cast<uint32_t>(ni), static_cast<uint32_t>(nl), 0u};
    memcpy(o, hdr, 40);
    memcpy(o + 40, &h.n_keys, 8);
    o += 48;
    for (uint64_t i = 0; i < ni; ++i) {
        memcpy(o, ik.data() + i * kSlots * kb, kSlots * kb);
        memset(o + kFirstSlot * kb, 0xFF, kb);  // the first-child slot is padding in the exported format
        memcpy(o + kSlots * kb, ic.data() + i * kSlots * 4, kSlots * 4);
        o += inner_rec_bytes(kb);
    }
    for (uint64_t i = 0; i < nl; ++i) {
        memcpy(o, lk.data() + i * kSlots * kb, kSlots * kb);
        memcpy(o + kSlots * kb, lv.data() + i * kSlots * kb, kSlots * kb);
        memcpy(o + 2 * kSlots * kb, lm.data() + i * 8, 8);
        o += leaf_rec_bytes(kb);
    }
    *bytes = need;
    return GT_OK;
}

}  // extern "C"
