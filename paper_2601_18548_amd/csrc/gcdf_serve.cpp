// Serving loop: continuous batching of gcdf_request on one device.
//
// Host side of the persistent serving kernel (serve_loop in gcdf_serve_kernel.hip):
//  * gcdf_submit queues a request and returns its ticket at once;
//  * a worker thread admits queued requests in FIFO order while a request slot
//    is free and the in-flight memory stays within the budget, writes each
//    one's descriptor into pinned host memory and publishes it;
//  * the persistent kernel (one workgroup per compute unit) claims tiles of
//    every published request, so requests that arrive while others run share
//    the device; after an idle period the whole grid exits together (a grid
//    that had lost part of its workgroups would keep serving at a fraction of
//    the device while new arrivals kept the rest busy) and the worker relaunches
//    it when work is pending;
//  * completion is a per-slot sequence number written by the device with a
//    system-scope release; gcdf_poll and the worker read it.
#include "gcdf_serve.h"

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace gcdf {

namespace {

constexpr int64_t kMaxQueued = 1 << 16;
constexpr uint64_t kIdleTicks = 200000;  // 2 ms of the 100 MHz real-time counter

// First-fit allocator of device scratch, in units of 8-byte keys.
class KeyPool {
 public:
  void init(int64_t n) { free_[0] = n; }
  int64_t alloc(int64_t n) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        const int64_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > n) free_[off + n] = len - n;
        return off;
      }
    }
    return -1;
  }
  void release(int64_t off, int64_t n) {
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

 private:
  std::map<int64_t, int64_t> free_;  // offset -> length
};

enum class TState { kQueued, kRunning, kDone };

struct Ticket {
  gcdf_request req;
  TState state = TState::kQueued;
  uint64_t seq = 0;
  size_t bytes = 0;
  int64_t key_off = -1;
};

size_t request_bytes(const gcdf_request& r, int obstacle_floats) {
  const size_t pairs = (size_t)r.K * (size_t)r.Np;
  size_t b = (size_t)r.K * 36 + (size_t)r.Np * 4 * obstacle_floats;
  if (r.d) b += pairs * 4;
  if (r.J) b += pairs * 36;
  if (r.dmin) b += (size_t)r.K * 16;  // dmin + argmin + key scratch
  if (r.Jmin) b += (size_t)r.K * 36;
  return b;
}

}  // namespace

struct Server {
  gcdf_ctx* ctx = nullptr;
  int device = 0;
  size_t budget = 0;
  uint32_t slots = 0;
  ServeCtl* ctl = nullptr;      // pinned host memory
  ServeDev* dev = nullptr;      // device memory
  unsigned long long* keys = nullptr;
  int64_t key_cap = 0;
  KeyPool pool;
  hipStream_t stream = nullptr;
  hipEvent_t kernel_done = nullptr;
  bool kernel_live = false;
  uint32_t epoch = 0;           // launches so far (the drain word starts at 0)

  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool quit = false;
  gcdf_status device_error = GCDF_OK;

  uint64_t next_ticket = 1;
  uint64_t next_seq = 0;
  size_t inflight_bytes = 0;
  std::deque<uint64_t> queue;                     // queued tickets, FIFO
  std::unordered_map<uint64_t, Ticket> tickets;
  std::map<uint64_t, uint64_t> running;           // seq -> ticket
  std::vector<uint64_t> slot_done_total;          // cumulative tiles per slot

  // Requests whose completion flag is set: release their slot and memory.
  void reap_locked() {
    for (auto it = running.begin(); it != running.end();) {
      const uint64_t seq = it->first;
      const uint64_t flag = __atomic_load_n(&ctl->complete[seq % slots], __ATOMIC_ACQUIRE);
      if (flag >= seq + 1) {
        Ticket& t = tickets[it->second];
        t.state = TState::kDone;
        inflight_bytes -= t.bytes;
        if (t.key_off >= 0) pool.release(t.key_off, t.req.K);
        it = running.erase(it);
      } else {
        ++it;
      }
    }
  }

  // Oldest request still running or queued-for-publication (the kernel's start cursor).
  uint64_t lowest_live_seq_locked() const { return running.empty() ? next_seq : running.begin()->first; }

  // Admit and publish queued requests while slots and memory allow.
  void admit_locked() {
    while (!queue.empty()) {
      Ticket& t = tickets[queue.front()];
      const uint64_t seq = next_seq;
      const uint32_t s = (uint32_t)(seq % slots);
      if (seq >= slots && running.count(seq - slots)) break;  // slot still busy
      if (inflight_bytes + t.bytes > budget) break;            // memory
      int64_t off = -1;
      if (t.req.dmin) {
        off = pool.alloc(t.req.K);
        if (off < 0) break;
      }
      const int64_t nblk = (t.req.Np + kTileQ - 1) / kTileQ;
      const int64_t ntiles = t.req.K * nblk;
      ServeDesc& d = ctl->desc[s];
      // seqlock: a device reader that sees the marker or another number knows the
      // slot's previous request has completed (reap_locked freed the slot)
      __atomic_store_n(&d.seq, kDescWriting, __ATOMIC_RELAXED);
      std::atomic_thread_fence(std::memory_order_release);  // marker before the fields
      d.knots = t.req.knots;
      d.points = t.req.points;
      d.K = t.req.K;
      d.Np = t.req.Np;
      d.nblk = nblk;
      d.ntiles = ntiles;
      slot_done_total[s] += (uint64_t)ntiles;
      d.done_target = slot_done_total[s];
      d.d = t.req.d;
      d.J = t.req.J;
      d.minkey = off >= 0 ? keys + off : nullptr;
      d.dmin = t.req.dmin;
      d.argmin = t.req.argmin;
      d.Jmin = t.req.Jmin;
      d.want_grad = t.req.J ? 1 : 0;
      __atomic_store_n(&d.seq, seq, __ATOMIC_RELEASE);  // fields before the number
      __atomic_store_n(&ctl->published, seq + 1, __ATOMIC_RELEASE);
      t.state = TState::kRunning;
      t.seq = seq;
      t.key_off = off;
      inflight_bytes += t.bytes;
      running[seq] = queue.front();
      queue.pop_front();
      ++next_seq;
    }
  }

  // Relaunch the persistent kernel if it has exited while work is published.
  void ensure_kernel_locked() {
    if (kernel_live) {
      const hipError_t q = hipEventQuery(kernel_done);
      if (q == hipErrorNotReady) return;
      kernel_live = false;
      if (q != hipSuccess) {
        device_error = GCDF_EDEVICE;
        return;
      }
    }
    if (running.empty()) return;
    if (++epoch == 0) ++epoch;
    const hipError_t e = launch_serve(ctx_net(ctx), ctl, dev, lowest_live_seq_locked(), kIdleTicks, epoch,
                                      ctx_num_cu(ctx), stream);
    if (e == hipSuccess && hipEventRecord(kernel_done, stream) == hipSuccess) {
      kernel_live = true;
    } else {
      device_error = GCDF_EDEVICE;
    }
  }

  void loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (!quit) {
      if (__atomic_load_n(&ctl->fault, __ATOMIC_ACQUIRE) != 0) device_error = GCDF_EDEVICE;
      reap_locked();
      admit_locked();
      if (device_error == GCDF_OK) ensure_kernel_locked();
      const bool busy = !running.empty() || !queue.empty();
      cv.wait_for(lk, busy ? std::chrono::microseconds(20) : std::chrono::milliseconds(5));
    }
  }
};

gcdf_status server_start(gcdf_ctx* ctx, size_t mem_budget, int nslots, Server** out) {
  if (nslots < 1 || nslots > kMaxSlots) return set_error(GCDF_EINVAL, "serve_slots must be in [1, 256]");
  Server* sv = new Server;
  sv->ctx = ctx;
  sv->device = ctx_device(ctx);
  sv->budget = mem_budget;
  sv->slots = (uint32_t)nslots;
  sv->slot_done_total.assign(nslots, 0);
  // key scratch: enough for the budget's worth of dmin requests, capped
  sv->key_cap = (int64_t)std::min<size_t>(mem_budget / 16 + 1, (size_t)1 << 24);
  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&sv->ctl), sizeof(ServeCtl), hipHostMallocCoherent);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&sv->dev), sizeof(ServeDev));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&sv->keys), sv->key_cap * 8);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&sv->kernel_done, hipEventDisableTiming);
  if (e == hipSuccess) {
    std::memset(sv->ctl, 0, sizeof(ServeCtl));
    sv->ctl->slots = sv->slots;
    e = hipMemsetAsync(sv->dev, 0, sizeof(ServeDev), sv->stream);
  }
  if (e == hipSuccess) e = launch_fill_ones(sv->keys, sv->key_cap, sv->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(sv->stream);
  if (e != hipSuccess) {
    server_stop(sv);
    return set_error(GCDF_ENOMEM, "serving setup failed");
  }
  sv->pool.init(sv->key_cap);
  sv->worker = std::thread([sv] { sv->loop(); });
  *out = sv;
  return GCDF_OK;
}

void server_stop(Server* sv) {
  if (!sv) return;
  if (sv->worker.joinable()) {
    // drain: every queued and running request completes first (bounded wait)
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      const auto deadline = std::chrono::steady_clock::now() + std::chrono::seconds(120);
      while ((!sv->queue.empty() || !sv->running.empty()) && sv->device_error == GCDF_OK &&
             std::chrono::steady_clock::now() < deadline) {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(100));
        lk.lock();
      }
      sv->quit = true;
      if (sv->ctl) __atomic_store_n(&sv->ctl->stop, 1u, __ATOMIC_RELEASE);
    }
    sv->cv.notify_all();
    sv->worker.join();
  }
  if (sv->stream) {
    (void)hipStreamSynchronize(sv->stream);
    (void)hipStreamDestroy(sv->stream);
  }
  if (sv->kernel_done) (void)hipEventDestroy(sv->kernel_done);
  (void)hipFree(sv->keys);
  (void)hipFree(sv->dev);
  if (sv->ctl) (void)hipHostFree(sv->ctl);
  delete sv;
}

gcdf_status server_submit(Server* sv, const gcdf_request* r, uint64_t* ticket) {
  if (!r->knots || !r->points) return set_error(GCDF_EINVAL, "request knots/points pointer is NULL");
  if (r->K <= 0 || r->Np <= 0) return set_error(GCDF_EINVAL, "request K and Np must be positive");
  if (r->K > INT64_MAX / 9 / r->Np) return set_error(GCDF_EINVAL, "request K*Np*9 overflows int64");
  if (!r->d && !r->J && !r->dmin) return set_error(GCDF_EINVAL, "request asks for no output");
  if ((r->dmin == nullptr) != (r->argmin == nullptr)) return set_error(GCDF_EINVAL, "dmin and argmin go together");
  if (r->Jmin && !r->dmin) return set_error(GCDF_EINVAL, "Jmin needs dmin and argmin");
  if (r->dmin && r->Np > INT32_MAX) return set_error(GCDF_EINVAL, "request Np exceeds 2^31-1");
  if (r->K * ((r->Np + kTileQ - 1) / kTileQ) >= ((int64_t)1 << 32)) return set_error(GCDF_EINVAL, "request too large");
  const size_t bytes = request_bytes(*r, ctx_net(sv->ctx).in_dim == kInDimSphere ? 4 : 3);
  if (bytes > sv->budget) return set_error(GCDF_ENOMEM, "request needs more memory than serve_mem_budget");
  if (r->dmin && r->K > sv->key_cap) return set_error(GCDF_ENOMEM, "request K exceeds the key scratch");
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->device_error != GCDF_OK) return set_error(sv->device_error, "serving stopped after a device error");
  if ((int64_t)sv->queue.size() >= kMaxQueued) return set_error(GCDF_EBUSY, "serving queue is full");
  const uint64_t id = sv->next_ticket++;
  Ticket t;
  t.req = *r;
  t.bytes = bytes;
  sv->tickets.emplace(id, t);
  sv->queue.push_back(id);
  sv->cv.notify_one();
  *ticket = id;
  return GCDF_OK;
}

gcdf_status server_poll(Server* sv, uint64_t ticket) {
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->tickets.find(ticket);
  if (it == sv->tickets.end()) return set_error(GCDF_EINVAL, "unknown ticket");
  if (it->second.state == TState::kRunning) sv->reap_locked();
  if (it->second.state == TState::kDone) {
    sv->tickets.erase(it);
    return GCDF_OK;
  }
  if (sv->device_error != GCDF_OK) return set_error(sv->device_error, "serving stopped after a device error");
  return GCDF_PENDING;
}

}  // namespace gcdf
