// Native serving loop: continuous batching of polynomial and integer products by HBM
// budget (the batching of section 2.2's Remark 6 applied to a request stream).
//
// Requests carry host operands.  progress() admits pending requests in arrival order
// while the device arena has room: consecutive polynomial requests form one batched call
// (polymul_modp_batch: one fused launch per size class), an integer product is one
// intmul_crt call.  Each batch owns one arena block [operands | products | workspace]
// and one page-locked staging block [operands | products], so a batch costs one upload,
// one library call and one download, all asynchronous on one of the server's streams,
// followed by an event.  Batches on different streams overlap on the device.  The host
// copies into and out of the staging blocks run on a pool of copy threads, and the
// driving thread never waits for them: a batch's operands are copied while earlier
// batches compute, it is enqueued by the first progress() call after its copy, and its
// products are copied out while later batches compute (one thread's memcpy is well
// below the host's memory bandwidth, and a loop that waited for the copies would leave
// the device idle meanwhile).  Not thread-safe: one host thread drives a server.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/ntt_mi355x.h"

namespace {

const size_t kAlign = 256;
size_t up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Req {
  uint64_t id;
  int kind;  // 0 polynomial product mod p, 1 integer product (16-bit limbs)
  uint64_t p;
  const void* a;
  size_t la;
  const void* b;
  size_t lb;
  void* c;
  bool direct;  // c is page-locked: the product goes there by DMA, not through staging
  size_t esz() const { return kind == 1 ? 2 : (p < (1ull << 31) ? 4 : 8); }
  size_t out_elems() const { return kind == 1 ? (la + lb + 1) / 2 : la + lb - 1; }
  size_t out_esz() const { return kind == 1 ? 4 : esz(); }
  size_t op_bytes() const { return up(la * esz()) + up(lb * esz()); }
  size_t out_bytes() const { return up(out_elems() * out_esz()); }
};

// First-fit allocator over [0, size) with coalescing.
struct Arena {
  std::map<size_t, size_t> free_;  // offset -> size
  size_t used = 0;
  explicit Arena(size_t size) { free_[0] = size; }
  bool alloc(size_t n, size_t* off) {
    n = up(std::max<size_t>(n, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const size_t rest = it->second - n;
      const size_t o = it->first;
      free_.erase(it);
      if (rest) free_[o + n] = rest;
      used += n;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = up(std::max<size_t>(n, 1));
    used -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

// Host copies split into 1 MiB pieces that the pool's threads take in turn.  submit()
// returns at once; a job's `done` runs on the thread that finishes its last piece.
class CopyPool {
 public:
  struct Copy {
    void* dst;
    const void* src;
    size_t n;
  };
  explicit CopyPool(int threads) {
    for (int i = 0; i < threads; ++i) th_.emplace_back([this] { worker(); });
  }
  ~CopyPool() {
    drain();
    {
      std::lock_guard<std::mutex> g(m_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  void submit(const std::vector<Copy>& jobs, std::function<void()> done) {
    static const size_t kPiece = 1u << 20;
    auto t = std::make_shared<Task>();
    for (const Copy& c : jobs)
      for (size_t o = 0; o < c.n; o += kPiece)
        t->p.push_back(Copy{(char*)c.dst + o, (const char*)c.src + o, std::min(kPiece, c.n - o)});
    if (t->p.empty() || th_.empty()) {  // nothing to copy, or no pool: on the caller
      for (const Copy& c : t->p) memcpy(c.dst, c.src, c.n);
      done();
      return;
    }
    t->left = t->p.size();
    t->done = std::move(done);
    {
      std::lock_guard<std::mutex> g(m_);
      q_.push_back(t);
      ++active_;
    }
    cv_.notify_all();
  }
  // Returns when every submitted job has completed (its `done` included).
  void drain() {
    std::unique_lock<std::mutex> lk(m_);
    idle_.wait(lk, [&] { return active_ == 0; });
  }

 private:
  struct Task {
    std::vector<Copy> p;
    size_t next = 0;  // next piece to hand out (under m_)
    std::atomic<size_t> left{0};
    std::function<void()> done;
  };
  void worker() {
    for (;;) {
      std::shared_ptr<Task> t;
      size_t i = 0;
      {
        std::unique_lock<std::mutex> lk(m_);
        cv_.wait(lk, [&] { return stop_ || !q_.empty(); });
        if (q_.empty()) return;  // stop_ with nothing queued
        t = q_.front();
        i = t->next++;
        if (t->next >= t->p.size()) q_.pop_front();
      }
      memcpy(t->p[i].dst, t->p[i].src, t->p[i].n);
      if (t->left.fetch_sub(1) == 1) {
        t->done();
        {
          std::lock_guard<std::mutex> g(m_);
          --active_;
        }
        idle_.notify_all();
      }
    }
  }
  std::vector<std::thread> th_;
  std::mutex m_;
  std::condition_variable cv_, idle_;
  std::deque<std::shared_ptr<Task>> q_;
  size_t active_ = 0;  // jobs submitted and not yet completed
  bool stop_ = false;
};

struct Staging {
  void* host = nullptr;
  size_t cap = 0;
  std::atomic<bool> busy{false};  // cleared by the copy thread that drains it
};

// A batch moves through: operands copied into its staging block (copy threads), then
// upload, library call, download and event enqueued (the driving thread), then its
// products copied out of staging (copy threads), then retired.
enum BatchState { kCopyIn = 0, kReady, kLaunched, kCopyOut, kDone };

struct Batch {
  std::vector<Req> reqs;
  std::vector<size_t> off_a, off_b, off_c;  // offsets inside the block (and staging)
  size_t op_bytes = 0, out_bytes = 0, ws_off = 0, ws_bytes = 0, block = 0, block_bytes = 0;
  Staging* stg = nullptr;  // its staging block (blocks never move: the copy threads use this)
  hipEvent_t ev = nullptr;
  std::atomic<int> state{kCopyIn};
};

}  // namespace

struct ntt_server {
  int device = 0;
  unsigned char* dbuf = nullptr;
  size_t budget = 0;
  Arena* arena = nullptr;
  std::vector<hipStream_t> streams;
  unsigned next_stream = 0;
  size_t max_batch = 64;
  // operand + product bytes of one polynomial batch (smaller batches: shorter tails); a
  // little over 32 MiB so that the largest single request of 2^20-word 64-bit operands
  // (8 + 8 + 16 MiB, plus alignment) fits without a block of its own
  size_t staging_cap = (32u << 20) + (1u << 16);
  std::deque<Staging> staging;  // a deque: growing it moves no block the copy threads use
  std::vector<hipEvent_t> free_events;
  std::deque<Req> pending;
  std::deque<std::shared_ptr<Batch>> inflight;  // admission order
  size_t max_inflight = 0;
  size_t inflight_cap = 8;  // batches in flight at once: 2 per stream, one staging block each
  CopyPool* pool = nullptr;
  std::mutex fin_m;
  std::deque<uint64_t> finished;  // completed requests not yet handed back (under fin_m)
};

namespace {

// Whether host memory at ptr is page-locked (hipHostMalloc, torch pin_memory): then
// a device-to-host copy can land there directly.  The query's error for pageable
// memory is cleared so that no later hipGetLastError reports it.
bool page_locked(const void* ptr) {
  if (!ptr) return false;
  hipPointerAttribute_t at;
  memset(&at, 0, sizeof(at));
  const hipError_t e = hipPointerGetAttributes(&at, ptr);
  (void)hipGetLastError();
  return e == hipSuccess && at.type == hipMemoryTypeHost;
}

int acquire_staging(ntt_server* s, size_t bytes, Staging** out) {
  for (Staging& st : s->staging) {
    if (!st.busy.load() && st.cap >= bytes) {
      st.busy = true;
      *out = &st;
      return NTT_OK;
    }
  }
  const size_t cap = std::max(bytes, s->staging_cap);
  void* host = nullptr;
  if (hipHostMalloc(&host, cap, hipHostMallocDefault) != hipSuccess) return NTT_ENOMEM;
  s->staging.emplace_back();
  s->staging.back().host = host;
  s->staging.back().cap = cap;
  s->staging.back().busy = true;
  *out = &s->staging.back();
  return NTT_OK;
}

// Layout of a batch and its device bytes (operands, products, library workspace).
int layout(Batch& bt) {
  size_t o = 0;
  bt.off_a.clear();
  bt.off_b.clear();
  bt.off_c.clear();
  for (const Req& r : bt.reqs) {
    bt.off_a.push_back(o);
    o += up(r.la * r.esz());
    bt.off_b.push_back(o);
    o += up(r.lb * r.esz());
  }
  bt.op_bytes = o;
  for (const Req& r : bt.reqs) {
    bt.off_c.push_back(o);
    o += r.out_bytes();
  }
  bt.out_bytes = o - bt.op_bytes;
  bt.ws_off = o;
  if (bt.reqs[0].kind == 1) {
    bt.ws_bytes = intmul_workspace_bytes(bt.reqs[0].la, bt.reqs[0].lb);
  } else {
    std::vector<ntt_polymul_desc> d(bt.reqs.size());
    for (size_t i = 0; i < bt.reqs.size(); ++i) {
      const Req& r = bt.reqs[i];
      // shapes only: any aligned pointers
      d[i] = ntt_polymul_desc{r.p, (const void*)(uintptr_t)4096, r.la, (const void*)(uintptr_t)4096, r.lb,
                              (void*)(uintptr_t)4096};
    }
    bt.ws_bytes = polymul_batch_workspace_bytes(d.data(), d.size());
  }
  bt.block_bytes = bt.ws_off + up(bt.ws_bytes);
  return NTT_OK;
}

// Operands into the batch's staging block, on the copy threads; the batch turns kReady.
int stage_in(ntt_server* s, const std::shared_ptr<Batch>& b) {
  Batch& bt = *b;
  int rc = acquire_staging(s, bt.op_bytes + bt.out_bytes, &bt.stg);
  if (rc) return rc;
  unsigned char* host = (unsigned char*)bt.stg->host;
  std::vector<CopyPool::Copy> cp;
  for (size_t i = 0; i < bt.reqs.size(); ++i) {
    const Req& r = bt.reqs[i];
    cp.push_back(CopyPool::Copy{host + bt.off_a[i], r.a, r.la * r.esz()});
    cp.push_back(CopyPool::Copy{host + bt.off_b[i], r.b, r.lb * r.esz()});
  }
  bt.state = kCopyIn;
  s->pool->submit(cp, [b] { b->state = kReady; });
  return NTT_OK;
}

// Upload, library call, download and event of a batch whose operands are staged.
int enqueue(ntt_server* s, Batch& bt) {
  int rc = NTT_OK;
  unsigned char* host = (unsigned char*)bt.stg->host;
  hipStream_t st = s->streams[s->next_stream++ % s->streams.size()];
  unsigned char* dev = s->dbuf + bt.block;
  if (hipMemcpyAsync(dev, host, bt.op_bytes, hipMemcpyHostToDevice, st) != hipSuccess) return NTT_EDEVICE;
  if (bt.reqs[0].kind == 1) {
    const Req& r = bt.reqs[0];
    rc = intmul_crt((const uint16_t*)(dev + bt.off_a[0]), r.la, (const uint16_t*)(dev + bt.off_b[0]), r.lb,
                    (uint32_t*)(dev + bt.off_c[0]), dev + bt.ws_off, bt.ws_bytes, st);
  } else {
    std::vector<ntt_polymul_desc> d(bt.reqs.size());
    for (size_t i = 0; i < bt.reqs.size(); ++i) {
      const Req& r = bt.reqs[i];
      d[i] = ntt_polymul_desc{r.p, dev + bt.off_a[i], r.la, dev + bt.off_b[i], r.lb, dev + bt.off_c[i]};
    }
    rc = polymul_modp_batch(d.data(), d.size(), bt.ws_bytes ? dev + bt.ws_off : nullptr, bt.ws_bytes, st);
  }
  if (rc) return rc;
  // products: page-locked destinations by DMA each, the others through staging (one copy
  // of the whole product region)
  bool staged = false;
  for (size_t i = 0; i < bt.reqs.size(); ++i) {
    const Req& r = bt.reqs[i];
    if (!r.c) continue;
    if (!r.direct) {
      staged = true;
      continue;
    }
    if (hipMemcpyAsync(r.c, dev + bt.off_c[i], r.out_elems() * r.out_esz(), hipMemcpyDeviceToHost, st) != hipSuccess)
      return NTT_EDEVICE;
  }
  if (staged && hipMemcpyAsync(host + bt.op_bytes, dev + bt.op_bytes, bt.out_bytes, hipMemcpyDeviceToHost, st) !=
                    hipSuccess)
    return NTT_EDEVICE;
  if (!bt.ev) {
    if (!s->free_events.empty()) {
      bt.ev = s->free_events.back();
      s->free_events.pop_back();
    } else if (hipEventCreateWithFlags(&bt.ev, hipEventDisableTiming) != hipSuccess) {
      return NTT_EDEVICE;
    }
  }
  if (hipEventRecord(bt.ev, st) != hipSuccess) return NTT_EDEVICE;
  return NTT_OK;
}

// Products of a batch finished on the device out of staging into the requests'
// buffers, on the copy threads; then the ids queue for hand-back and the staging block
// is free again.
void stage_out(ntt_server* s, const std::shared_ptr<Batch>& b) {
  const Batch& bt = *b;
  const unsigned char* host = (const unsigned char*)bt.stg->host;
  std::vector<CopyPool::Copy> cp;
  for (size_t i = 0; i < bt.reqs.size(); ++i) {
    const Req& r = bt.reqs[i];
    if (r.c && !r.direct) cp.push_back(CopyPool::Copy{r.c, host + bt.off_c[i], r.out_elems() * r.out_esz()});
  }
  b->state = kCopyOut;
  s->pool->submit(cp, [s, b] {
    {
      std::lock_guard<std::mutex> g(s->fin_m);
      for (const Req& r : b->reqs) s->finished.push_back(r.id);
    }
    b->stg->busy = false;
    b->state = kDone;
  });
}

}  // namespace

extern "C" {

int ntt_server_create(ntt_server** out, size_t hbm_budget, int streams, size_t max_batch) {
  if (!out || hbm_budget == 0 || streams < 1 || streams > 16 || max_batch < 1) return NTT_EINVAL;
  *out = nullptr;
  ntt_server* s = new (std::nothrow) ntt_server();
  if (!s) return NTT_ENOMEM;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return NTT_EDEVICE;
  }
  if (hipMalloc((void**)&s->dbuf, hbm_budget) != hipSuccess) {
    delete s;
    return NTT_ENOMEM;
  }
  s->budget = hbm_budget;
  s->arena = new Arena(hbm_budget);
  {
    // copy threads besides the calling one: the tuning choice server.copy_threads, else 7
    // (bounded by the host's hardware threads)
    const unsigned hw = std::thread::hardware_concurrency();
    int64_t want = 7;
    if (ntt_tune_get("server.copy_threads", &want) != NTT_OK) want = 7;
    s->pool = new CopyPool((int)std::min<int64_t>(want, hw > 1 ? hw - 1 : 0));
  }
  s->max_batch = max_batch;
  for (int i = 0; i < streams; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {  // default priority
      ntt_server_destroy(s);
      return NTT_EDEVICE;
    }
    s->streams.push_back(st);
  }
  // page-locked staging allocated once (its allocation is slow), one block per batch in
  // flight (a batch holds its block from the operands' copy until its products are out);
  // batches in flight per stream: the tuning choice server.batches_per_stream, else 2
  int64_t per_stream = 2;
  if (ntt_tune_get("server.batches_per_stream", &per_stream) != NTT_OK) per_stream = 2;
  s->inflight_cap = (size_t)per_stream * (size_t)streams;
  for (size_t i = 0; i < s->inflight_cap; ++i) {
    void* host = nullptr;
    if (hipHostMalloc(&host, s->staging_cap, hipHostMallocDefault) != hipSuccess) {
      ntt_server_destroy(s);
      return NTT_ENOMEM;
    }
    s->staging.emplace_back();
    s->staging.back().host = host;
    s->staging.back().cap = s->staging_cap;
  }
  *out = s;
  return NTT_OK;
}

int ntt_server_destroy(ntt_server* s) {
  if (!s) return NTT_OK;
  for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
  if (s->pool) s->pool->drain();  // no copy may touch staging or requests after this
  for (auto& b : s->inflight)
    if (b->ev) (void)hipEventDestroy(b->ev);
  for (hipEvent_t e : s->free_events) (void)hipEventDestroy(e);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  for (Staging& st : s->staging)
    if (st.host) (void)hipHostFree(st.host);
  if (s->dbuf) (void)hipFree(s->dbuf);
  delete s->pool;
  delete s->arena;
  delete s;
  return NTT_OK;
}

int ntt_server_submit(ntt_server* s, uint64_t id, int kind, uint64_t p, const void* a, size_t la, const void* b,
                      size_t lb, void* c) {
  if (!s || !a || !b || la == 0 || lb == 0 || (kind != 0 && kind != 1)) return NTT_EINVAL;
  if (kind == 0) {
    if (p < 3 || p >= (1ull << 62) || !ntt_is_prime(p)) return NTT_ENOTPRIME;
    int L = 0;
    while (((size_t)1 << L) < la + lb - 1) ++L;
    if (((p - 1) & (((uint64_t)1 << L) - 1)) != 0 || L > 26) return NTT_ENOROOT;
  } else if (la + lb - 1 > ((size_t)1 << 23)) {
    return NTT_EINVAL;
  }
  Req r{id, kind, p, a, la, b, lb, c, page_locked(c)};
  Batch one;
  one.reqs.push_back(r);
  layout(one);
  if (one.block_bytes > s->budget) return NTT_ENOMEM;  // never fits, even alone
  s->pending.push_back(r);
  return NTT_OK;
}

namespace {

// A batch that could not be enqueued: nothing of it is pending on the device once the
// streams are drained; its memory goes back and its requests to the front of the queue.
void give_back(ntt_server* s, const std::shared_ptr<Batch>& b) {
  for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
  if (b->stg) b->stg->busy = false;
  if (b->ev) s->free_events.push_back(b->ev);
  b->ev = nullptr;
  s->arena->release(b->block, b->block_bytes);
  for (size_t i = b->reqs.size(); i-- > 0;) s->pending.push_front(b->reqs[i]);
  for (auto it = s->inflight.begin(); it != s->inflight.end(); ++it)
    if (*it == b) {
      s->inflight.erase(it);
      break;
    }
}

}  // namespace

int ntt_server_progress(ntt_server* s, uint64_t* done_ids, size_t cap, size_t* ndone) {
  if (!s || !ndone || (cap && !done_ids)) return NTT_EINVAL;
  *ndone = 0;
  // (1) device side: batches whose operands are staged are enqueued; batches whose work
  // has finished give their memory back to the arena and start their copy-out
  for (size_t k = 0; k < s->inflight.size(); ++k) {
    std::shared_ptr<Batch> b = s->inflight[k];
    const int st = b->state.load();
    if (st == kReady) {
      const int rc = enqueue(s, *b);
      if (rc) {
        give_back(s, b);
        return rc;
      }
      b->state = kLaunched;
    } else if (st == kLaunched) {
      const hipError_t q = hipEventQuery(b->ev);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return NTT_EDEVICE;
      s->arena->release(b->block, b->block_bytes);
      stage_out(s, b);
    }
  }
  // (2) retire batches whose products are out (their ids are already queued)
  for (auto it = s->inflight.begin(); it != s->inflight.end();) {
    if ((*it)->state.load() == kDone) {
      s->free_events.push_back((*it)->ev);
      it = s->inflight.erase(it);
    } else {
      ++it;
    }
  }
  // (3) admissions in arrival order: operands start their copy into staging
  while (!s->pending.empty() && s->inflight.size() < s->inflight_cap) {
    auto b = std::make_shared<Batch>();
    Batch& bt = *b;
    if (s->pending.front().kind == 1) {
      bt.reqs.push_back(s->pending.front());
    } else {
      size_t staged = 0;
      for (const Req& r : s->pending) {
        if (r.kind != 0 || bt.reqs.size() >= s->max_batch) break;
        const size_t nb = r.op_bytes() + r.out_bytes();
        if (!bt.reqs.empty() && staged + nb > s->staging_cap) break;
        bt.reqs.push_back(r);
        staged += nb;
      }
    }
    // shrink the batch until its block fits in the arena
    bool placed = false;
    while (!bt.reqs.empty()) {
      layout(bt);
      if (s->arena->alloc(bt.block_bytes, &bt.block)) {
        placed = true;
        break;
      }
      bt.reqs.pop_back();
    }
    if (!placed) break;  // wait for memory to free up
    for (size_t i = 0; i < bt.reqs.size(); ++i) s->pending.pop_front();
    s->inflight.push_back(b);
    const int rc = stage_in(s, b);
    if (rc) {
      give_back(s, b);
      return rc;
    }
    s->max_inflight = std::max(s->max_inflight, s->inflight.size());
  }
  {
    std::lock_guard<std::mutex> g(s->fin_m);
    while (*ndone < cap && !s->finished.empty()) {
      done_ids[(*ndone)++] = s->finished.front();
      s->finished.pop_front();
    }
  }
  return NTT_OK;
}

int ntt_server_stats(const ntt_server* s, size_t* pending, size_t* inflight, size_t* arena_used, size_t* max_inflight) {
  if (!s) return NTT_EINVAL;
  if (pending) *pending = s->pending.size();
  if (inflight) {
    // batches not yet retired whose products are still on the way, plus completed
    // requests not yet handed back
    size_t live = 0;
    for (const auto& b : s->inflight) live += b->state.load() != kDone;
    std::lock_guard<std::mutex> g(const_cast<ntt_server*>(s)->fin_m);
    *inflight = live + s->finished.size();
  }
  if (arena_used) *arena_used = s->arena->used;
  if (max_inflight) *max_inflight = s->max_inflight;
  return NTT_OK;
}

}  // extern "C"
