// Serving runtime: continuous batching of lookup / insert / range batches
// over one resident tree (and optional learned index).
//
// One worker thread owns every HIP call of the server.  Each pass it
//   1. retires finished batches (event query), copies their outputs from
//      pinned staging to the caller's buffers and frees slot and bytes;
//  1b. with a learned index and retrain_log2 set: once 2^retrain_log2 keys
//      were inserted since training, what training reads of the tree (child
//      references, leaf keys and metadata in use) is copied on the write
//      stream (after the writes admitted so far, before any admitted later;
//      reads go on) and a trainer thread trains a second index against the
//      copy on its own stream, masked to a few CUs, while admission
//      continues.  The trained index
//      is bound to the live tree with the copy's insert and delete counts,
//      so the lookups treat every later write as a change since training
//      (a miss is then checked along the leaf chain or the tree, as for any
//      index that inserts made stale).  At the next pass after training the
//      worker exchanges its state with the serving index's: batches
//      admitted from then on use it (their lookup graphs are captured again),
//      batches already launched keep the state they were launched with, and
//      the old state is not trained into again until every batch admitted
//      before the exchange has retired;
//   2. admits queued batches in arrival order while a slot is free and the
//      staged bytes in flight stay under the cap (a batch larger than the
//      cap is refused at once, so admission never deadlocks);
//   3. launches each admitted batch: inputs are copied into the slot's
//      pinned buffers, padded to a power of two with entries that leave the
//      result unchanged, then the slot's captured graph for (op, size) is
//      replayed -- or captured on first use -- on a stream chosen by the
//      op: reads spread over several streams, inserts on one write stream.
// Ordering: admission order is the linearization order.  A read waits for
// the last admitted insert (a dedicated event re-recorded on the write
// stream); an insert waits for every read admitted since the previous
// insert.  Reads therefore overlap reads, and every batch's result equals
// its result when the batches run one at a time in admission order.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/gtree.h"
#include "common.h"
#include "handle.h"

namespace {

using clk = std::chrono::steady_clock;

// The trainer's stream runs on 32 of the 256 CUs, four per XCD (bit i of
// the mask selects a CU of XCD i mod 8), so a retraining leaves the rest of
// the GPU to the batches being served.
constexpr uint32_t kTrainCuMaskWords = 8;
const uint32_t kTrainCuMask[kTrainCuMaskWords] = {0xFFFFFFFFu, 0, 0, 0, 0, 0, 0, 0};

double now_s() {
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

uint32_t pow2ceil(uint64_t x) {
    uint32_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

struct Req {
    gt_request r;
    double arrival;
    double done;
    uint32_t state;
    uint32_t slot;
    uint64_t bytes;
    bool failed;
    float dev0 = -1.0f, dev1 = -1.0f;  // device start / end (ms after the replay's reference event)
};

struct Slot {
    bool busy = false;
    uint64_t ticket = 0;
    hipEvent_t ev = nullptr;   // recorded after the batch's work (completion, end time)
    hipEvent_t ev0 = nullptr;  // recorded before it (start time)
    // device staging
    uint8_t* d_keys = nullptr; uint8_t* d_vals = nullptr; uint32_t* d_max = nullptr; uint64_t* d_off = nullptr;
    uint8_t* d_out0 = nullptr; uint8_t* d_out1 = nullptr; uint32_t* d_cnt = nullptr; uint8_t* d_flag = nullptr;
    // pinned host staging
    uint8_t* h_keys = nullptr; uint8_t* h_vals = nullptr; uint32_t* h_max = nullptr; uint64_t* h_off = nullptr;
    uint8_t* h_out0 = nullptr; uint8_t* h_out1 = nullptr; uint32_t* h_cnt = nullptr; uint8_t* h_flag = nullptr;
    uint32_t* h_err = nullptr;
    std::map<uint64_t, hipGraphExec_t> graphs;
    uint64_t li_gen = 0;   // learned-index generation the lookup graphs were captured at
    // lookup graphs the trainer captured for a retrained index, installed at
    // the exchange when the index's state still matches (next_flags)
    std::map<uint64_t, hipGraphExec_t> next_graphs;
    uint64_t next_flags = 0;
    uint32_t bucket = 0;
    uint64_t out_len = 0;  // staged range output entries
};

}  // namespace

struct gt_server {
    gt_tree* t = nullptr;
    gt_learned* li = nullptr;
    gt_srv_params p{};
    int kb = 8;
    std::vector<Slot> slots;
    std::vector<hipStream_t> rstreams;
    hipStream_t wstream = nullptr, cstream = nullptr;
    hipEvent_t wev = nullptr;
    hipEvent_t ref_ev = nullptr;          // device time origin of the current replay
    bool ref_set = false;
    uint64_t replay_first = UINT64_MAX;   // first ticket of the current replay
    bool have_write = false;
    std::vector<hipEvent_t> reads_since_write;
    uint32_t rr = 0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::deque<Req> reqs;
    std::thread worker;
    std::atomic<bool> stop{false};
    uint64_t bytes_inflight = 0;
    uint32_t inflight = 0;
    uint64_t graph_launches = 0, direct_launches = 0;
    uint64_t captures = 0, precaptured = 0;
    double capture_s = 0.0;
    hipStream_t tcstream = nullptr;     // the trainer's capture stream
    uint64_t inserted_since_train = 0;  // keys of completed insert batches since the last retrain
    bool retrain_due = false;           // enough keys inserted: retrain when the spare state is free
    // retraining beside the serving index
    int device = 0;
    gt_learned* shadow = nullptr;       // trained on a copy of the tree, then exchanged with li
    void* shadow_arena = nullptr;
    uint8_t* snap_arena = nullptr;      // the copy of the tree's arena
    gt_tree* snap = nullptr;            // a handle over the copy
    hipStream_t tstream = nullptr;      // the trainer's stream
    hipEvent_t snap_ev = nullptr;       // recorded after the copy on the write stream
    std::thread trainer;
    bool train_running = false;         // copy and training under way
    bool shadow_ready = false;          // trained: exchange at the next pass
    gt_status train_status = GT_OK;
    uint64_t snap_inserts = 0, snap_deletes = 0;
    uint64_t exchange_ticket = 0;       // batches admitted before the last exchange have smaller tickets
    void* user_arena = nullptr;         // the caller's index arena (its state returns there at the end)
    double train_t0 = 0.0;
    uint64_t retrains = 0;
    double retrain_s = 0.0;
    std::vector<uint64_t> last_replay;
    hipError_t fatal = hipSuccess;
};

namespace {

uint64_t staged_bytes(const gt_server* s, const gt_request& r, uint32_t bucket, uint64_t outn) {
    const uint64_t kb = s->kb;
    switch (r.op) {
        case GT_OP_LOOKUP: return bucket * (2 * kb + 1);
        case GT_OP_INSERT: return bucket * (2 * kb + 1);
        case GT_OP_DELETE: return bucket * (kb + 1);
        default: return bucket * (2 * kb + 4 + 8 + 4) + outn * 2 * kb;
    }
}

uint64_t range_total(const gt_request& r) {
    uint64_t tot = 0;
    for (uint32_t i = 0; i < r.B; ++i) tot += r.max_out[i];
    return tot;
}

// Fill the slot's pinned inputs for request r padded to `bucket`.
void stage_inputs(gt_server* s, Slot& sl, const gt_request& r, uint32_t bucket, uint64_t outn) {
    const uint64_t kb = s->kb;
    memcpy(sl.h_keys, r.keys, r.B * kb);
    if (r.op == GT_OP_LOOKUP) {
        // padding repeats the last key: its answers are ignored, and it takes
        // the path of a real query (an absent filler key would make every
        // padded batch of a stale learned index descend the tree for it)
        for (uint32_t i = r.B; i < bucket; ++i) memcpy(sl.h_keys + i * kb, sl.h_keys + (r.B - 1) * kb, kb);
    } else if (r.op == GT_OP_INSERT) {
        memcpy(sl.h_vals, r.values, r.B * kb);
        // padding repeats the last pair: same final value, statuses ignored
        for (uint32_t i = r.B; i < bucket; ++i) {
            memcpy(sl.h_keys + i * kb, sl.h_keys + (r.B - 1) * kb, kb);
            memcpy(sl.h_vals + i * kb, sl.h_vals + (r.B - 1) * kb, kb);
        }
    } else if (r.op == GT_OP_DELETE) {
        // padding repeats the last key: deleted once, statuses ignored
        for (uint32_t i = r.B; i < bucket; ++i) memcpy(sl.h_keys + i * kb, sl.h_keys + (r.B - 1) * kb, kb);
    } else {
        memcpy(sl.h_vals, r.values, r.B * kb);
        uint64_t off = 0;
        for (uint32_t i = 0; i < bucket; ++i) {
            if (i < r.B) {
                sl.h_max[i] = r.max_out[i];
            } else {
                // an empty interval (lo = 1 > hi = 0) with max 0
                memset(sl.h_keys + i * kb, 0, kb);
                sl.h_keys[i * kb] = 1;
                memset(sl.h_vals + i * kb, 0, kb);
                sl.h_max[i] = 0;
            }
            sl.h_off[i] = off;
            off += sl.h_max[i];
        }
        (void)outn;
    }
}

// Enqueue the whole batch (copies in, kernels, copies out) on stream st.
hipError_t enqueue_ops(gt_server* s, Slot& sl, uint32_t op, uint32_t bucket, uint64_t outn, hipStream_t st,
                       gt_learned* li) {
    const uint64_t kb = s->kb;
    hipError_t e;
    if ((e = hipMemcpyAsync(sl.d_keys, sl.h_keys, bucket * kb, hipMemcpyHostToDevice, st)) != hipSuccess) return e;
    if (op == GT_OP_LOOKUP) {
        gt_status g = li ? li_lookup_batch(li, sl.d_keys, bucket, sl.d_out0, sl.d_flag, st)
                            : tree_lookup_batch(s->t, sl.d_keys, bucket, sl.d_out0, sl.d_flag, st);
        if (g != GT_OK) return hipErrorUnknown;
        if ((e = hipMemcpyAsync(sl.h_out0, sl.d_out0, bucket * kb, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(sl.h_flag, sl.d_flag, bucket, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    } else if (op == GT_OP_INSERT) {
        if ((e = hipMemcpyAsync(sl.d_vals, sl.h_vals, bucket * kb, hipMemcpyHostToDevice, st)) != hipSuccess) return e;
        // this batch reports only its own outcome
        gt::launch_clear_error(s->t->hdr, st);
        if (tree_insert_batch(s->t, sl.d_keys, sl.d_vals, bucket, sl.d_flag, st) != GT_OK) return hipErrorUnknown;
        if ((e = hipMemcpyAsync(sl.h_flag, sl.d_flag, bucket, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(sl.h_err, &s->t->hdr->error, 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    } else if (op == GT_OP_DELETE) {
        gt::launch_clear_error(s->t->hdr, st);
        if (tree_delete_batch(s->t, sl.d_keys, bucket, sl.d_flag, st) != GT_OK) return hipErrorUnknown;
        if ((e = hipMemcpyAsync(sl.h_flag, sl.d_flag, bucket, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(sl.h_err, &s->t->hdr->error, 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    } else {
        if ((e = hipMemcpyAsync(sl.d_vals, sl.h_vals, bucket * kb, hipMemcpyHostToDevice, st)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(sl.d_max, sl.h_max, bucket * 4, hipMemcpyHostToDevice, st)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(sl.d_off, sl.h_off, bucket * 8, hipMemcpyHostToDevice, st)) != hipSuccess) return e;
        if (tree_range_batch(s->t, sl.d_keys, sl.d_vals, sl.d_max, sl.d_off, bucket, sl.d_out0, sl.d_out1, sl.d_cnt,
                             st) != GT_OK)
            return hipErrorUnknown;
        if ((e = hipMemcpyAsync(sl.h_cnt, sl.d_cnt, bucket * 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
        if (outn) {
            if ((e = hipMemcpyAsync(sl.h_out0, sl.d_out0, outn * kb, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
            if ((e = hipMemcpyAsync(sl.h_out1, sl.d_out1, outn * kb, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// Capture the batch's work on stream cs (thread-local capture mode, so other
// threads keep launching) and instantiate it.
hipError_t capture_ops(gt_server* s, Slot& sl, uint32_t op, uint32_t bucket, uint64_t outn, hipStream_t cs,
                       gt_learned* li, hipGraphExec_t* out) {
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t e2 = enqueue_ops(s, sl, op, bucket, outn, cs, li);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    if (e2 != hipSuccess) {
        if (g) hipGraphDestroy(g);
        return e2;
    }
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    return e;
}

hipError_t launch(gt_server* s, Slot& sl, uint32_t op, uint32_t bucket, uint64_t outn, hipStream_t st) {
    const bool graphs = s->p.use_graphs != 2;
    if (!graphs || op == GT_OP_DELETE) {  // a delete waits on the host: never captured
        s->direct_launches++;
        return enqueue_ops(s, sl, op, bucket, outn, st, s->li);
    }
    if (op == GT_OP_LOOKUP && s->li) {
        // a retrained (or re-bounded) learned index: its lookup graphs are stale
        const uint64_t gen = gt_li_generation(s->li);
        if (gen != sl.li_gen) {
            for (auto g = sl.graphs.begin(); g != sl.graphs.end();) {
                if ((g->first >> 56) == GT_OP_LOOKUP) {
                    hipGraphExecDestroy(g->second);
                    g = sl.graphs.erase(g);
                } else {
                    ++g;
                }
            }
            sl.li_gen = gen;
        }
    }
    const uint64_t key = (static_cast<uint64_t>(op) << 56) | (static_cast<uint64_t>(bucket) << 28) | outn;
    auto it = sl.graphs.find(key);
    if (it == sl.graphs.end()) {
        const double t0 = now_s();
        hipGraphExec_t x = nullptr;
        hipError_t e = capture_ops(s, sl, op, bucket, outn, s->cstream, s->li, &x);
        if (e != hipSuccess) return e;
        s->captures++;
        s->capture_s += now_s() - t0;
        it = sl.graphs.emplace(key, x).first;
    }
    s->graph_launches++;
    return hipGraphLaunch(it->second, st);
}

// Copy the finished batch's outputs to the caller.
void retire(gt_server* s, Slot& sl, Req& q) {
    const gt_request& r = q.r;
    const uint64_t kb = s->kb;
    if (r.op == GT_OP_LOOKUP) {
        memcpy(r.out0, sl.h_out0, r.B * kb);
        memcpy(r.out1, sl.h_flag, r.B);
    } else if (r.op == GT_OP_INSERT || r.op == GT_OP_DELETE) {
        memcpy(r.out0, sl.h_flag, r.B);
        q.failed = *sl.h_err != 0;
    } else {
        memcpy(r.count_out, sl.h_cnt, r.B * 4);
        uint64_t tot = 0;
        for (uint32_t i = 0; i < r.B; ++i) tot += r.max_out[i];
        memcpy(r.out0, sl.h_out0, tot * kb);
        memcpy(r.out1, sl.h_out1, tot * kb);
    }
}

// Capture, for the retrained index, the lookup graphs every slot holds now,
// so that the worker does not capture them again after the exchange.  The
// captures only record the slots' buffers (no work runs); the worker keeps
// launching meanwhile.  Graphs are tagged with the index's stale / deleted
// state, which decides the lookup kernel: at the exchange they are used only
// if that state has not moved on.
void precapture(gt_server* s) {
    std::vector<std::vector<uint64_t>> keys(s->slots.size());
    {
        std::lock_guard<std::mutex> g(s->mu);
        for (size_t i = 0; i < s->slots.size(); ++i) {
            for (auto& kv : s->slots[i].next_graphs) hipGraphExecDestroy(kv.second);
            s->slots[i].next_graphs.clear();
            for (auto& kv : s->slots[i].graphs)
                if ((kv.first >> 56) == GT_OP_LOOKUP) keys[i].push_back(kv.first);
        }
    }
    const uint64_t flags = gt_li_generation(s->shadow) & 3u;
    for (size_t i = 0; i < s->slots.size(); ++i) {
        std::map<uint64_t, hipGraphExec_t> made;
        for (uint64_t k : keys[i]) {
            const uint32_t bucket = static_cast<uint32_t>((k >> 28) & ((1u << 28) - 1));
            hipGraphExec_t x = nullptr;
            if (capture_ops(s, s->slots[i], GT_OP_LOOKUP, bucket, 0, s->tcstream, s->shadow, &x) != hipSuccess) break;
            made.emplace(k, x);
        }
        std::lock_guard<std::mutex> g(s->mu);
        s->slots[i].next_graphs.swap(made);
        s->slots[i].next_flags = flags;
    }
}

// The trainer thread: train the shadow index against the copy of the tree
// on its own stream, bind it to the live tree, and hand it to the worker.
void trainer_run(gt_server* s) {
    gt_status st = hipSetDevice(s->device) == hipSuccess ? GT_OK : GT_ERR_HIP;
    if (st == GT_OK && hipStreamWaitEvent(s->tstream, s->snap_ev, 0) != hipSuccess) st = GT_ERR_HIP;
    if (st == GT_OK) {
        gt_li_rebind(s->shadow, s->snap, 0, 0);
        st = li_train(s->shadow, s->tstream);
        gt_li_rebind(s->shadow, s->t, s->snap_inserts, s->snap_deletes);
    }
    if (st == GT_OK && s->p.use_graphs != 2) precapture(s);
    std::lock_guard<std::mutex> g(s->mu);
    s->train_status = st;
    s->shadow_ready = true;
    s->cv_work.notify_all();
}

void worker_loop(gt_server* s) {
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        bool did = false;
        // 1. retire finished batches
        for (uint32_t i = 0; i < s->slots.size(); ++i) {
            Slot& sl = s->slots[i];
            if (!sl.busy) continue;
            if (hipEventQuery(sl.ev) != hipSuccess) continue;
            Req& q = s->reqs[sl.ticket];
            retire(s, sl, q);
            // deleted keys count too: after a delete the index answers
            // through the tree until it is trained again
            if ((q.r.op == GT_OP_INSERT || q.r.op == GT_OP_DELETE) && !q.failed && s->shadow) {
                s->inserted_since_train += q.r.B;
                if (s->inserted_since_train >= (1ull << s->p.retrain_log2)) s->retrain_due = true;
            }
            if (s->ref_set) {
                float a = 0, b = 0;
                if (hipEventElapsedTime(&a, s->ref_ev, sl.ev0) == hipSuccess &&
                    hipEventElapsedTime(&b, s->ref_ev, sl.ev) == hipSuccess) {
                    q.dev0 = a;
                    q.dev1 = b;
                }
            }
            q.done = now_s();
            q.state = q.failed ? GT_REQ_REFUSED : GT_REQ_DONE;
            s->bytes_inflight -= q.bytes;
            s->inflight--;
            sl.busy = false;
            did = true;
        }
        if (did) s->cv_done.notify_all();
        // 1b. retraining beside the serving index: exchange a trained shadow
        //     state, or start the next training once enough keys were
        //     inserted and no batch still runs on the spare state
        if (s->shadow_ready) {
            if (s->trainer.joinable()) s->trainer.join();
            if (s->train_status == GT_OK) {
                gt_li_exchange(s->li, s->shadow);
                s->exchange_ticket = s->queue.empty() ? s->reqs.size() : s->queue.front();
                s->retrains++;
                // the trainer's graphs replace the slots' lookup graphs when
                // the index's state is the one they were captured for
                const uint64_t gen = gt_li_generation(s->li);
                for (Slot& sl : s->slots) {
                    if (sl.next_graphs.empty() || sl.next_flags != (gen & 3u)) continue;
                    for (auto g = sl.graphs.begin(); g != sl.graphs.end();) {
                        if ((g->first >> 56) == GT_OP_LOOKUP) {
                            hipGraphExecDestroy(g->second);
                            g = sl.graphs.erase(g);
                        } else {
                            ++g;
                        }
                    }
                    for (auto& kv : sl.next_graphs) sl.graphs.emplace(kv.first, kv.second);
                    s->precaptured += sl.next_graphs.size();
                    sl.next_graphs.clear();
                    sl.li_gen = gen;
                }
            } else {
                s->fatal = hipErrorUnknown;
            }
            s->retrain_s += now_s() - s->train_t0;
            s->shadow_ready = false;
            s->train_running = false;
            s->cv_done.notify_all();
            did = true;
        }
        if (s->retrain_due && !s->train_running && s->fatal == hipSuccess) {
            bool spare_busy = false;
            for (const Slot& sl : s->slots)
                if (sl.busy && sl.ticket < s->exchange_ticket) spare_busy = true;
            if (!spare_busy) {
                // the copy reads the tree between the writes admitted so far
                // and any admitted later (both on the write stream)
                hipError_t e = gt_tree_copy_for_training(s->t, s->snap, s->wstream) == GT_OK ? hipSuccess
                                                                                              : hipErrorUnknown;
                if (e == hipSuccess) e = hipEventRecord(s->snap_ev, s->wstream);
                if (e != hipSuccess) {
                    s->fatal = e;
                } else {
                    s->snap_inserts = s->t->inserts;
                    s->snap_deletes = s->t->deletes;
                    s->inserted_since_train = 0;
                    s->retrain_due = false;
                    s->train_running = true;
                    s->train_t0 = now_s();
                    if (s->trainer.joinable()) s->trainer.join();
                    s->trainer = std::thread(trainer_run, s);
                }
                did = true;
            }
        }
        // 2. admit in arrival order
        while (!s->queue.empty() && s->fatal == hipSuccess) {
            const uint64_t tk = s->queue.front();
            Req& q = s->reqs[tk];
            const uint32_t bucket = pow2ceil(q.r.B ? q.r.B : 1);
            const uint64_t outn = q.r.op == GT_OP_RANGE ? pow2ceil(range_total(q.r) + 1) : 0;
            const uint64_t need = staged_bytes(s, q.r, bucket, outn);
            if (need > s->p.mem_cap) {
                s->queue.pop_front();
                q.state = GT_REQ_REFUSED;
                q.done = now_s();
                s->cv_done.notify_all();
                continue;
            }
            if (s->bytes_inflight + need > s->p.mem_cap) break;
            uint32_t free_slot = UINT32_MAX;
            for (uint32_t i = 0; i < s->slots.size(); ++i)
                if (!s->slots[i].busy) { free_slot = i; break; }
            if (free_slot == UINT32_MAX) break;
            s->queue.pop_front();
            Slot& sl = s->slots[free_slot];
            stage_inputs(s, sl, q.r, bucket, outn);
            hipStream_t st;
            const bool write = q.r.op == GT_OP_INSERT || q.r.op == GT_OP_DELETE;
            if (write) {
                st = s->wstream;
                for (hipEvent_t e : s->reads_since_write) hipStreamWaitEvent(st, e, 0);
                s->reads_since_write.clear();
            } else {
                st = s->rstreams[s->rr++ % s->rstreams.size()];
                if (s->have_write) hipStreamWaitEvent(st, s->wev, 0);
            }
            hipError_t e = hipSuccess;
            if (tk == s->replay_first) {
                e = hipEventRecord(s->ref_ev, st);
                s->ref_set = e == hipSuccess;
            }
            if (e == hipSuccess) e = hipEventRecord(sl.ev0, st);
            if (e == hipSuccess) e = launch(s, sl, q.r.op, bucket, outn, st);
            if (e == hipSuccess) e = hipEventRecord(sl.ev, st);
            if (e == hipSuccess && write) {
                e = hipEventRecord(s->wev, st);
                s->have_write = true;
            } else if (e == hipSuccess) {
                s->reads_since_write.push_back(sl.ev);
            }
            if (e != hipSuccess) {
                s->fatal = e;
                q.state = GT_REQ_REFUSED;
                q.done = now_s();
                s->cv_done.notify_all();
                continue;
            }
            sl.busy = true;
            sl.ticket = tk;
            q.slot = free_slot;
            q.bytes = need;
            q.state = GT_REQ_INFLIGHT;
            s->bytes_inflight += need;
            s->inflight++;
            did = true;
        }
        if (s->fatal != hipSuccess && !s->queue.empty()) {
            // a launch failed: nothing more is admitted, so refuse what waits
            for (uint64_t tk : s->queue) {
                s->reqs[tk].state = GT_REQ_REFUSED;
                s->reqs[tk].done = now_s();
            }
            s->queue.clear();
            s->cv_done.notify_all();
        }
        if (s->stop && s->queue.empty() && s->inflight == 0) break;
        if (s->inflight == 0 && s->queue.empty()) {
            s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
        } else if (!did) {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        }
    }
}

gt_status alloc_slot(gt_server* s, Slot& sl) {
    const uint64_t B = s->p.max_batch, kb = s->kb, R = static_cast<uint64_t>(s->p.max_batch) * s->p.max_range + 1;
    const uint64_t outn = pow2ceil(R);
    auto dm = [](void** p, uint64_t n) { return hipMalloc(p, n ? n : 1) == hipSuccess; };
    auto hm = [](void** p, uint64_t n) { return hipHostMalloc(p, n ? n : 1, hipHostMallocDefault) == hipSuccess; };
    bool ok = dm((void**)&sl.d_keys, B * kb) && dm((void**)&sl.d_vals, B * kb) && dm((void**)&sl.d_max, B * 4) &&
              dm((void**)&sl.d_off, B * 8) && dm((void**)&sl.d_out0, std::max(B, outn) * kb) &&
              dm((void**)&sl.d_out1, std::max(B, outn) * kb) && dm((void**)&sl.d_cnt, B * 4) &&
              dm((void**)&sl.d_flag, B) && hm((void**)&sl.h_keys, B * kb) && hm((void**)&sl.h_vals, B * kb) &&
              hm((void**)&sl.h_max, B * 4) && hm((void**)&sl.h_off, B * 8) &&
              hm((void**)&sl.h_out0, std::max(B, outn) * kb) && hm((void**)&sl.h_out1, std::max(B, outn) * kb) &&
              hm((void**)&sl.h_cnt, B * 4) && hm((void**)&sl.h_flag, B) && hm((void**)&sl.h_err, 4);
    if (!ok) return GT_ERR_HIP;
    // timing events: the device-busy fraction is measured from them
    if (hipEventCreate(&sl.ev) != hipSuccess || hipEventCreate(&sl.ev0) != hipSuccess) return GT_ERR_HIP;
    return GT_OK;
}

void free_slot(Slot& sl) {
    for (auto& kv : sl.graphs) hipGraphExecDestroy(kv.second);
    sl.graphs.clear();
    for (auto& kv : sl.next_graphs) hipGraphExecDestroy(kv.second);
    sl.next_graphs.clear();
    if (sl.ev) hipEventDestroy(sl.ev);
    if (sl.ev0) hipEventDestroy(sl.ev0);
    void* d[] = {sl.d_keys, sl.d_vals, sl.d_max, sl.d_off, sl.d_out0, sl.d_out1, sl.d_cnt, sl.d_flag};
    for (void* p : d)
        if (p) hipFree(p);
    void* h[] = {sl.h_keys, sl.h_vals, sl.h_max, sl.h_off, sl.h_out0, sl.h_out1, sl.h_cnt, sl.h_flag, sl.h_err};
    for (void* p : h)
        if (p) hipHostFree(p);
}

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (v.size() - 1);
    const size_t i = static_cast<size_t>(pos);
    const double f = pos - i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

gt_status submit_at(gt_server* s, const gt_request* r, double arrival, uint64_t* ticket) {
    if (!s || !r || !ticket) return GT_ERR_INVALID;
    if (r->op > GT_OP_DELETE || r->B == 0 || r->B > s->p.max_batch || !r->keys || !r->out0) return GT_ERR_INVALID;
    if ((r->op == GT_OP_LOOKUP && !r->out1) || ((r->op == GT_OP_INSERT || r->op == GT_OP_RANGE) && !r->values) ||
        (r->op == GT_OP_RANGE && (!r->max_out || !r->out1 || !r->count_out)))
        return GT_ERR_INVALID;
    if (r->op == GT_OP_RANGE)
        for (uint32_t i = 0; i < r->B; ++i)
            if (r->max_out[i] > s->p.max_range) return GT_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->fatal != hipSuccess) return GT_ERR_HIP;
    Req q;
    q.r = *r;
    q.arrival = arrival;
    q.done = 0;
    q.state = GT_REQ_QUEUED;
    q.slot = 0;
    q.bytes = 0;
    q.failed = false;
    s->reqs.push_back(q);
    const uint64_t tk = s->reqs.size() - 1;
    s->queue.push_back(tk);
    *ticket = tk;
    s->cv_work.notify_one();
    return GT_OK;
}

}  // namespace

extern "C" {

gt_status srv_create(gt_tree* t, gt_learned* li, const gt_srv_params* p, gt_server** out) {
    if (!t || t->wide || !out) return GT_ERR_INVALID;
    gt_srv_params q{};
    if (p) q = *p;
    if (q.use_graphs > 2 || q.retrain_log2 > 40) return GT_ERR_INVALID;
    if (!q.read_streams) q.read_streams = 4;
    if (!q.slots) q.slots = 16;
    if (!q.mem_cap) q.mem_cap = 32ull << 30;
    if (!q.max_batch) q.max_batch = 1024;
    if (!q.max_range) q.max_range = 128;
    if (!q.use_graphs) q.use_graphs = 1;
    if (q.max_batch > t->max_batch || q.read_streams > 64 || q.slots > 256) return GT_ERR_INVALID;
    gt_server* s = new gt_server();
    s->t = t;
    s->li = li;
    s->p = q;
    s->kb = t->kb;
    s->slots.resize(q.slots);
    gt_status st = GT_OK;
    for (Slot& sl : s->slots)
        if ((st = alloc_slot(s, sl)) != GT_OK) break;
    if (st == GT_OK) {
        s->rstreams.resize(q.read_streams);
        for (auto& x : s->rstreams)
            if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess) st = GT_ERR_HIP;
        if (hipStreamCreateWithFlags(&s->wstream, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&s->cstream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s->wev, hipEventDisableTiming) != hipSuccess ||
            hipEventCreate(&s->ref_ev) != hipSuccess)
            st = GT_ERR_HIP;
    }
    if (st == GT_OK && li && q.retrain_log2) {
        // the second index and the tree copy it trains on, allocated now
        const uint64_t lb = gt_li_arena_bytes_like(li);
        s->user_arena = gt_li_arena(li);
        if (hipGetDevice(&s->device) != hipSuccess || hipMalloc(&s->shadow_arena, lb) != hipSuccess ||
            hipMalloc(reinterpret_cast<void**>(&s->snap_arena), t->arena_bytes) != hipSuccess ||
            hipExtStreamCreateWithCUMask(&s->tstream, kTrainCuMaskWords, kTrainCuMask) != hipSuccess ||
            hipStreamCreateWithFlags(&s->tcstream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s->snap_ev, hipEventDisableTiming) != hipSuccess)
            st = GT_ERR_HIP;
        if (st == GT_OK) st = gt_li_create_like(li, s->shadow_arena, lb, &s->shadow);
        if (st == GT_OK) s->snap = gt_tree_clone_handle(t, s->snap_arena);
    }
    if (st != GT_OK) {
        srv_destroy(s);
        return st;
    }
    // the tree was built on another stream: make sure it is complete
    if (hipDeviceSynchronize() != hipSuccess) {
        srv_destroy(s);
        return GT_ERR_HIP;
    }
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return GT_OK;
}

gt_status srv_submit(gt_server* s, const gt_request* r, uint64_t* ticket) {
    return submit_at(s, r, now_s(), ticket);
}

gt_status srv_poll(gt_server* s, uint64_t ticket, uint32_t* state) {
    if (!s || !state) return GT_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    if (ticket >= s->reqs.size()) return GT_ERR_INVALID;
    *state = s->reqs[ticket].state;
    return GT_OK;
}

gt_status srv_wait(gt_server* s, uint64_t ticket) {
    if (!s) return GT_ERR_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    if (ticket >= s->reqs.size()) return GT_ERR_INVALID;
    s->cv_done.wait(lk, [&] {
        const uint32_t st = s->reqs[ticket].state;
        return st == GT_REQ_DONE || st == GT_REQ_REFUSED;
    });
    if (s->fatal != hipSuccess) return GT_ERR_HIP;
    return s->reqs[ticket].state == GT_REQ_DONE ? GT_OK : GT_ERR_ADMISSION;
}

gt_status srv_replay(gt_server* s, const gt_request* reqs, uint64_t n) {
    if (!s || (n && !reqs)) return GT_ERR_INVALID;
    std::vector<uint64_t> tickets(n);
    {
        // the worker records the device time origin when it admits this
        // replay's first request
        std::lock_guard<std::mutex> lk(s->mu);
        s->replay_first = s->reqs.size();
        s->ref_set = false;
    }
    const double t0 = now_s();
    for (uint64_t i = 0; i < n; ++i) {
        const double at = t0 + reqs[i].arrival_s;
        while (now_s() < at) {
            if (at - now_s() > 200e-6) std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
        gt_status st = submit_at(s, &reqs[i], at, &tickets[i]);
        if (st != GT_OK) return st;
    }
    gt_status res = GT_OK;
    for (uint64_t i = 0; i < n; ++i) {
        gt_status st = srv_wait(s, tickets[i]);
        if (st == GT_ERR_HIP) return st;
        if (st != GT_OK) res = GT_ERR_ADMISSION;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    // a retraining these inserts started is part of the replay
    s->cv_done.wait(lk, [&] { return (!s->retrain_due && !s->train_running) || s->fatal != hipSuccess; });
    s->last_replay = tickets;
    return res;
}

gt_status srv_stats(gt_server* s, gt_srv_stats* out) {
    if (!s || !out) return GT_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    memset(out, 0, sizeof *out);
    std::vector<double> all, per[4];
    std::vector<std::pair<float, float>> busy;
    double first = 1e300, last = 0;
    const std::vector<uint64_t>& ids = s->last_replay;
    for (uint64_t tk : ids) {
        const Req& q = s->reqs[tk];
        if (q.state == GT_REQ_REFUSED) {
            out->refused++;
            continue;
        }
        if (q.state != GT_REQ_DONE) continue;
        const double us = (q.done - q.arrival) * 1e6;
        all.push_back(us);
        per[q.r.op].push_back(us);
        out->done[q.r.op]++;
        out->ops[q.r.op] += q.r.B;
        first = std::min(first, q.arrival);
        last = std::max(last, q.done);
        if (q.dev1 >= q.dev0 && q.dev0 > -1.0f) busy.emplace_back(q.dev0, q.dev1);
    }
    out->graph_launches = s->graph_launches;
    out->direct_launches = s->direct_launches;
    out->captures = s->captures;
    out->capture_s = s->capture_s;
    out->precaptured = s->precaptured;
    out->retrains = s->retrains;
    out->retrain_s = s->retrain_s;
    out->wall_s = all.empty() ? 0.0 : last - first;
    out->p50_us = percentile(all, 0.5);
    out->p99_us = percentile(all, 0.99);
    for (int o = 0; o < 4; ++o) {
        out->p50_us_op[o] = percentile(per[o], 0.5);
        out->p99_us_op[o] = percentile(per[o], 0.99);
    }
    // union of the batches' device intervals over the wall time
    std::sort(busy.begin(), busy.end());
    double covered_ms = 0, cur0 = 0, cur1 = -1e300;
    for (const auto& iv : busy) {
        if (iv.first > cur1) {
            if (cur1 > cur0) covered_ms += cur1 - cur0;
            cur0 = iv.first;
            cur1 = iv.second;
        } else if (iv.second > cur1) {
            cur1 = iv.second;
        }
    }
    if (cur1 > cur0) covered_ms += cur1 - cur0;
    out->busy_frac = out->wall_s > 0 ? covered_ms * 1e-3 / out->wall_s : 0.0;
    return GT_OK;
}

gt_status srv_latencies(gt_server* s, double* out, uint64_t n) {
    if (!s || (n && !out)) return GT_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    if (n > s->last_replay.size()) return GT_ERR_INVALID;
    for (uint64_t i = 0; i < n; ++i) {
        const Req& q = s->reqs[s->last_replay[i]];
        out[i] = q.state == GT_REQ_DONE ? (q.done - q.arrival) * 1e6 : -1.0;
    }
    return GT_OK;
}

gt_status srv_destroy(gt_server* s) {
    if (!s) return GT_ERR_INVALID;
    if (s->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
            s->cv_work.notify_all();
        }
        s->worker.join();
    }
    if (s->trainer.joinable()) s->trainer.join();
    hipDeviceSynchronize();
    if (s->shadow) {
        // a training that finished after the last pass is still handed over
        if (s->shadow_ready && s->train_status == GT_OK) {
            gt_li_exchange(s->li, s->shadow);
            s->retrains++;
        }
        // the caller's index keeps its own arena: after an odd number of
        // exchanges its state sits in the server's arena and moves back
        if (gt_li_arena(s->li) != s->user_arena) {
            const uint64_t lb = gt_li_arena_bytes_like(s->li);
            if (hipMemcpy(s->user_arena, gt_li_arena(s->li), lb, hipMemcpyDeviceToDevice) == hipSuccess)
                gt_li_swap_arenas(s->li, s->shadow);
        }
        li_destroy(s->shadow);
    }
    if (s->shadow_arena) hipFree(s->shadow_arena);
    if (s->snap_arena) hipFree(s->snap_arena);
    delete s->snap;
    if (s->tstream) hipStreamDestroy(s->tstream);
    if (s->tcstream) hipStreamDestroy(s->tcstream);
    if (s->snap_ev) hipEventDestroy(s->snap_ev);
    for (Slot& sl : s->slots) free_slot(sl);
    for (auto x : s->rstreams)
        if (x) hipStreamDestroy(x);
    if (s->wstream) hipStreamDestroy(s->wstream);
    if (s->cstream) hipStreamDestroy(s->cstream);
    if (s->wev) hipEventDestroy(s->wev);
    if (s->ref_ev) hipEventDestroy(s->ref_ev);
    delete s;
    return GT_OK;
}

}  // extern "C"
