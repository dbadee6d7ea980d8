// Level-wise batch lookup (paper Sections IV-A and IV-F).
//
// The paper walks a sorted batch through the tree one level at a time.  A
// FIFO holds (node, number of queries) entries; each node is read once and
// compared with the run of consecutive sorted queries that passes through
// it, and the queries of that run that go to the same child form one entry
// of the next level.  Here the batch is sorted by the library (or arrives
// sorted from the caller), and each tree level is one kernel.
//
// The FIFO of a level is kept per window of 64 consecutive sorted queries.
// A run never crosses a window boundary (the root's run is cut at every
// window, and a child's run is a piece of its parent's), so each window's
// entries are described by a 64-bit mask with bit p set where a run starts
// at query p of the window, plus the node reference of each run stored at
// its first query's position.  No counter, scan or atomic is needed to
// append entries, and the order of the entries is the order of the keys.
//
//   * A wave serves a window, one lane per query.  The lane finds its run
//     (the nearest run start at or below it), reads the run's node
//     reference, and reads the node's key line with 16-byte loads.  All
//     lanes of a run load the same addresses in the same instructions, so
//     the memory system fetches the line once per run: the node is read
//     once and compared with every query of its run, the queries in
//     parallel rather than one after another as on the FPGA.
//   * Where the child differs from the previous query's, a new run starts;
//     its child reference and start bit go to the next level's FIFO.
//   * At the leaf level each lane matches its query in the leaf's key line
//     (read with the value line, once per run) and writes the result to the
//     query's position in the caller's order.
//
// What differs from the FPGA design: the root's run is cut at every window
// (so 256 CUs share the work); the root and the nodes near it are then read
// once per window, from the top-levels mirror (up to three levels, cached on
// chip), and the first kernel walks those levels itself, so their FIFOs
// never go through memory.  Unsorted queries still
// get correct answers: runs are only cut more often.  The host launches one
// kernel per level up to a bound on the height; a kernel whose level lies
// below the leaves (per the device header) returns at once.
#include <mutex>

#include "common.h"
#include "kernels.h"
#include "prims.h"
#include "traverse.h"

namespace gt {

constexpr int kLwBlock = 256;
constexpr int kLwWaves = kLwBlock / 64;
constexpr uint32_t kLwWin = 64;                 // queries per window (one wave)
constexpr uint32_t kLwGridMax = 2048;           // 8 resident workgroups per CU

// One tree level over every window of the batch.  Otherwise the runs of
// window w start at the set bits of hm_in[w], with their node references in
// ref_in at the runs' first positions.  ROOT: each window is one run through
// the root, and the levels the top-levels mirror holds (the root and up to
// two below it, cached on chip) are walked by every lane through the mirror
// in this kernel, which writes the FIFO of the first level below them (in
// hm_in/ref_in when that level is even, the buffers that level reads);
// the kernels of the mirrored levels then return at once.  Every lane of a
// wave stays active through the level (the cross-lane reads need their
// source lanes).
template <class K, bool ROOT>
__global__ __launch_bounds__(kLwBlock) void k_lw_level(TreeView<K> t, const K* __restrict__ qs,
                                                        const uint32_t* __restrict__ qi, uint32_t B, uint32_t level,
                                                        uint64_t* hm_in, uint32_t* ref_in,
                                                        uint64_t* __restrict__ hm_out, uint32_t* __restrict__ ref_out,
                                                        K* __restrict__ vout, uint8_t* __restrict__ fout) {
    const uint32_t height = t.hdr->height;
    if (level >= height) return;  // the whole grid: the tree has no such level
    using ML = MirrorLayout<K>;
    const uint32_t top = reinterpret_cast<const MirrorHeader*>(t.mirror)->levels;  // mirrored inner levels
    if (!ROOT && level < top) return;  // walked through the mirror by the first kernel
    const bool leaves = level + 1 == height;
    const bool empty = t.hdr->n_keys == 0;
    const uint32_t root = t.hdr->root;
    const int lane = lane_id();
    const uint32_t nwin = (B + kLwWin - 1) / kLwWin;
    const uint32_t waves = gridDim.x * kLwWaves;
    for (uint32_t w = blockIdx.x * kLwWaves + threadIdx.x / 64; w < nwin; w += waves) {
        const uint64_t w0 = static_cast<uint64_t>(w) * kLwWin;
        const uint32_t nq = B - static_cast<uint32_t>(w0) < kLwWin ? B - static_cast<uint32_t>(w0) : kLwWin;
        const bool valid = static_cast<uint32_t>(lane) < nq;
        const K key = valid ? qs[w0 + lane] : K(0);
        uint32_t ref = root;
        if (ROOT && top > 0) {
            // the mirrored levels, one lane per query (a window's lanes
            // mostly read the same mirror lines)
            const K* mkeys = reinterpret_cast<const K*>(t.mirror + ML::keys_off());
            const uint32_t* mchild = reinterpret_cast<const uint32_t*>(t.mirror + ML::child_off(kMirrorMaxNodes));
            const uint32_t* mfirst = reinterpret_cast<const uint32_t*>(t.mirror + ML::first_off(kMirrorMaxNodes));
            uint32_t m = 0;
            for (uint32_t lv = 0; lv < top; ++lv) {
                K sep[kSlots];
                load_vec<K, kSlots>(mkeys + static_cast<uint64_t>(m) * kSlots, sep);
                uint32_t ci = 0;
#pragma unroll
                for (int j = 0; j < kFirstSlot; ++j) ci += sep[j] < key ? 1u : 0u;
                ref = mchild[static_cast<uint64_t>(m) * kSlots + ci];
                if (lv + 1 < top) m = mfirst[m] + ci;
            }
            const uint32_t prev = shfl_u32(ref, lane > 0 ? lane - 1 : 0);
            const bool head = valid && (lane == 0 || ref != prev);
            const uint64_t Hn = __ballot(head);
            uint64_t* ho = (top & 1) ? hm_out : hm_in;
            uint32_t* ro = (top & 1) ? ref_out : ref_in;
            if (head) ro[w0 + lane] = ref;
            if (lane == 0) ho[w] = Hn;
            continue;
        }
        if (!ROOT) {
            // this query's run starts at the highest run start <= lane (a
            // lane past the window's end takes the last run: every lane
            // reads a real node of this level)
            const uint64_t H = hm_in[w];
            const uint64_t upto = lane < 63 ? (H & ((2ull << lane) - 1ull)) : H;
            const uint32_t start = 63u - static_cast<uint32_t>(__builtin_clzll(upto | 1ull));
            ref = ref_in[w0 + start];
        }
        if (leaves) {
            const uint64_t line = static_cast<uint64_t>(ref & ~kLeafTag) * kSlots;
            K lk[kSlots], lv[kSlots];
            load_vec<K, kSlots>(t.lkeys + line, lk);
            load_vec<K, kSlots>(t.lvals + line, lv);
            // slots past the leaf's count repeat its last key, so the first
            // equal slot is the key's own
            uint32_t slot = kSlots;
#pragma unroll
            for (int j = kSlots - 1; j >= 0; --j)
                if (lk[j] == key) slot = static_cast<uint32_t>(j);
            K v = kmax<K>();
#pragma unroll
            for (int j = 0; j < kSlots; ++j)
                if (slot == static_cast<uint32_t>(j)) v = lv[j];
            const bool hit = slot < kSlots && !empty;
            if (valid) {
                const uint32_t o = qi ? qi[w0 + lane] : static_cast<uint32_t>(w0) + static_cast<uint32_t>(lane);
                vout[o] = hit ? v : kmax<K>();
                fout[o] = hit ? 1 : 0;  // a miss is all ones with found = 0 (Section IV-D)
            }
        } else {
            K sep[kSlots];
            load_vec<K, kSlots>(t.ikeys + static_cast<uint64_t>(ref) * kSlots, sep);
            // child index = separators below the key ("key <= entry"
            // routing); slot 15 is never a separator: it holds the first
            // child reference of a node with consecutive children, else the
            // largest key
            uint32_t ci = 0;
#pragma unroll
            for (int j = 0; j < kFirstSlot; ++j) ci += sep[j] < key ? 1u : 0u;
            const K first = sep[kFirstSlot];
            uint32_t r;
            if (first != kmax<K>()) r = static_cast<uint32_t>(first) + ci;
            else r = t.ichild[static_cast<uint64_t>(ref) * kSlots + ci];
            const uint32_t prev = shfl_u32(r, lane > 0 ? lane - 1 : 0);
            const bool head = valid && (lane == 0 || r != prev);
            const uint64_t Hn = __ballot(head);
            if (head) ref_out[w0 + lane] = r;
            if (lane == 0) hm_out[w] = Hn;
        }
    }
}

// ------------------------------------------------------------ host side

static uint64_t lw_align(uint64_t x) { return (x + 255) / 256 * 256; }

LwLayout lw_layout(uint64_t B, int key_bytes, bool presorted) {
    LwLayout L{};
    const uint64_t n = B ? B : 1;
    const uint64_t nw = (n + kLwWin - 1) / kLwWin;
    uint64_t o = 0;
    L.ha = o;  o += lw_align(nw * 8);
    L.hb = o;  o += lw_align(nw * 8);
    L.ra = o;  o += lw_align(n * 4);
    L.rb = o;  o += lw_align(n * 4);
    if (!presorted) {
        L.sk = o;  o += lw_align(n * key_bytes);
        L.si = o;  o += lw_align(n * 4);
        if (n > kRankSortMax) {
            L.sk2 = o;  o += lw_align(n * key_bytes);
            L.si2 = o;  o += lw_align(n * 4);
            L.tmp = o;  o += lw_align(sort_tmp_bytes(n, key_bytes));
        }
    }
    L.total = o;
    return L;
}

template <class K>
void launch_lookup_levelwise(const TreeView<K>& t, const K* keys, uint64_t B, bool presorted, uint32_t levels,
                             K* vout, uint8_t* fout, void* ws, hipStream_t s) {
    const LwLayout L = lw_layout(B, sizeof(K), presorted);
    uint8_t* w = reinterpret_cast<uint8_t*>(ws);
    uint64_t* ha = reinterpret_cast<uint64_t*>(w + L.ha);
    uint64_t* hb = reinterpret_cast<uint64_t*>(w + L.hb);
    uint32_t* ra = reinterpret_cast<uint32_t*>(w + L.ra);
    uint32_t* rb = reinterpret_cast<uint32_t*>(w + L.rb);
    const uint32_t b = static_cast<uint32_t>(B);
    const K* qs = keys;
    const uint32_t* qi = nullptr;
    if (!presorted) {
        K* sk = reinterpret_cast<K*>(w + L.sk);
        uint32_t* si = reinterpret_cast<uint32_t*>(w + L.si);
        if (B <= kRankSortMax) {
            rank_sort_small<K>(keys, b, sk, si, nullptr, 0, s);
        } else {
            sort_from<K>(keys, sk, si, reinterpret_cast<K*>(w + L.sk2), reinterpret_cast<uint32_t*>(w + L.si2), B,
                         w + L.tmp, s, &t.hdr->error, kErrInternal);
        }
        qs = sk;
        qi = si;
    }
    const uint64_t nwin = (B + kLwWin - 1) / kLwWin;
    const uint64_t wgs = (nwin + kLwBlock / 64 - 1) / (kLwBlock / 64);
    const uint32_t grid = static_cast<uint32_t>(wgs < kLwGridMax ? wgs : kLwGridMax);
    for (uint32_t l = 0; l < levels; ++l) {
        uint64_t* hin = (l & 1) ? ha : hb;
        uint32_t* rin = (l & 1) ? ra : rb;
        uint64_t* hout = (l & 1) ? hb : ha;
        uint32_t* rout = (l & 1) ? rb : ra;
        if (l == 0)
            hipLaunchKernelGGL((k_lw_level<K, true>), dim3(grid), dim3(kLwBlock), 0, s, t, qs, qi, b, l, hin, rin,
                               hout, rout, vout, fout);
        else
            hipLaunchKernelGGL((k_lw_level<K, false>), dim3(grid), dim3(kLwBlock), 0, s, t, qs, qi, b, l, hin,
                               rin, hout, rout, vout, fout);
    }
}

template void launch_lookup_levelwise<uint32_t>(const TreeView<uint32_t>&, const uint32_t*, uint64_t, bool,
                                                uint32_t, uint32_t*, uint8_t*, void*, hipStream_t);
template void launch_lookup_levelwise<uint64_t>(const TreeView<uint64_t>&, const uint64_t*, uint64_t, bool,
                                                uint32_t, uint64_t*, uint8_t*, void*, hipStream_t);

// ---------------------------------------- allocation-free variant's scratch

// The workspace of the allocation-free level-wise lookup: a fixed array in
// device memory, one copy per GPU the library runs on, held until the
// process ends.  Host code never passes `scratch` itself to a kernel (on the
// host the name is only a stand-in for the device symbol); it passes the
// address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint8_t scratch[kLwScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];
}  // namespace

hipError_t lw_scratch(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        // the device is current: this resolves its own copy of the array
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace gt
