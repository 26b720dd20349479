// Persistent serving kernel (continuous batching of gcdf_request) for gfx950.
#include "gcdf_tile.h"

namespace gcdf {
// ----------------------------------------------------------------------------
// Persistent serving kernel.  Requests are published by the host in sequence
// order into ServeCtl (pinned host memory); every workgroup walks the sequence
// with its own cursor and claims tiles from the slot's (seq, count) word (a
// compare-and-swap re-tags it for a new request, a fetch_add hands out the
// rest), so a late workgroup can never run tiles of a request that has since
// been replaced in its slot under the wrong descriptor (descriptors are read
// seqlock-style, see desc_ntiles).  The first workgroup
// that stays idle ends the launch for all (the drain word); tiles not yet
// claimed then wait in the claim words for the next launch.
//
// Memory ordering is paid per request, not per tile: claims are relaxed; a
// workgroup acquires (system scope) once when it sees new publications; when it
// leaves a request (its next claim finds no tile left) it releases its output
// stores at agent scope once and adds the number of tiles it ran to the slot's
// done counter.  The workgroup whose addition completes the request acquires,
// decodes the per-knot minimum, restores the key scratch and publishes
// completion with a system-scope release store.  (Acquire and release at agent
// or system scope invalidate or write back the L2, which per tile would evict
// the packed weights.)
// ----------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T sys_relaxed(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Tile count of request `want` from its slot's descriptor, read seqlock-style:
// the descriptor's seq before and after the read must both be `want`.  Returns
// false if the slot no longer holds `want` (it has completed and the host is
// rewriting or has rewritten the slot for a later request).
__device__ __forceinline__ bool desc_ntiles(const ServeDesc* d, uint64_t want, int64_t& nt) {
  const uint64_t a = sys_relaxed(&d->seq);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");  // system scope: the field read follows
  nt = sys_relaxed(&d->ntiles);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");  // the field read precedes the re-check
  const uint64_t b = sys_relaxed(&d->seq);
  return a == want && b == want;
}

template <int W, int MODE, bool SPH>
__global__ __launch_bounds__((Geo<W, MODE>::THREADS), 1) void serve_loop(const DevNet net, ServeCtl* ctl, ServeDev* dev,
                                                          uint64_t first_seq, uint64_t idle_ticks, uint32_t epoch) {
  __shared__ __attribute__((aligned(16))) char lds[Geo<W, MODE>::LDS_BYTES];
  __shared__ int64_t claim_info[3];  // claimed seq (or -1: exit, -2: none), tile, seq to finalize (or -1)
  __shared__ ServeDesc cur;          // the request this workgroup is working on
  __shared__ ServeDesc fin;          // a request this workgroup completes
  __shared__ uint32_t ovf;
  TileCtx<W, MODE> tc(lds, &ovf, net, threadIdx.x);
  const int tid = threadIdx.x;
  uint64_t seq = first_seq;  // this workgroup's cursor in the request sequence
  uint64_t cur_seq = ~0ull;
  uint64_t idle_since = __builtin_amdgcn_s_memrealtime();
  const uint32_t slots = sys_relaxed(&ctl->slots);
  // thread 0's view of the queue
  uint64_t pub = 0, nt_seq = ~0ull;
  int64_t ntiles = 0;
  uint64_t open_count = 0;  // tiles of request cur_seq run here and not yet reported
  int backoff = 1;
  while (true) {
    if (tid == 0) {
      int64_t got_seq = -1, got_tile = 0, fin_seq = -1;
      bool leave = false;
      // Report the tiles of request cur_seq run here (the caller has established that
      // no further tile of it will be claimed here); the report that completes the
      // request makes this workgroup its finalizer.
      auto report = [&]() {
        const uint32_t s = (uint32_t)(cur_seq % slots);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // this workgroup's stores and atomics
        const unsigned long long done =
            __hip_atomic_fetch_add(&dev->done[s], open_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + open_count;
        open_count = 0;
        if (done == cur.done_target) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // every contributor's results
          fin = cur;
          fin_seq = (int64_t)cur_seq;
        }
      };
      while (true) {
        if (__hip_atomic_load(&dev->drain, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch) {
          // another workgroup ended this launch: claim nothing more
          if (open_count) report();
          leave = true;
          break;
        }
        if (seq >= pub) {
          const uint64_t p = sys_relaxed(&ctl->published);
          if (p > pub) {
            pub = p;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");  // system scope: the new descriptors
          }
        }
        if (seq < pub) {
          const uint32_t s = (uint32_t)(seq % slots);
          if (nt_seq != seq) {
            // A cursor behind the others can reach a request that has completed and
            // whose slot the host has already given to a later request: the
            // descriptor then describes that later request, and its tile count must
            // not be taken for seq's.
            if (!desc_ntiles(&ctl->desc[s], seq, ntiles)) {
              if (open_count && cur_seq == seq) report();  // (none: seq is complete)
              ++seq;
              if (fin_seq >= 0) break;
              continue;
            }
            nt_seq = seq;
          }
          // Claim word of the slot: (request tag << 32) | tiles handed out.  The first
          // claimant of a request re-tags the word with a compare-and-swap; every other
          // claim is a fetch_add, which never has to be retried.
          unsigned long long v = __hip_atomic_load(&dev->claim[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const uint64_t s32 = seq & 0xffffffffull;
          bool moved_on = false;
          while (true) {
            const uint64_t vs = v >> 32, vc = v & 0xffffffffull;
            if (vs > s32) { moved_on = true; break; }  // slot already reused: seq is complete
            if (vs < s32) {                            // first claim of request seq
              if (__hip_atomic_compare_exchange_strong(&dev->claim[s], &v, (s32 << 32) | 1ull, __ATOMIC_RELAXED,
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                got_seq = (int64_t)seq;
                got_tile = 0;
                break;
              }
              continue;  // v now holds the current word
            }
            if ((int64_t)vc >= ntiles) { moved_on = true; break; }
            const unsigned long long w =
                __hip_atomic_fetch_add(&dev->claim[s], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t ws = w >> 32, wc = w & 0xffffffffull;
            if (ws == s32) {
              if ((int64_t)wc < ntiles) { got_seq = (int64_t)seq; got_tile = (int64_t)wc; }
              else moved_on = true;
              break;
            }
            // Between the load and the add, request seq finished and a later request
            // took the slot: the add handed out tile wc of that request, which must be
            // run here.  Its tag is the low half of its sequence number.
            const uint64_t later = seq + ((ws - s32) & 0xffffffffull);
            // (no tiles of seq can be unreported here: seq could not have completed)
            seq = later;
            if (pub < later + 1) pub = later + 1;
            int64_t lnt = 0;
            bool held = false;
            // The request that tagged the word was published before its first claim,
            // so its descriptor is in place; a read that misses it is a visibility
            // delay, re-read (bounded).  A slot holding a newer request means `later`
            // has completed, so all its tiles were handed out: wc is past them.
            for (int tries = 0; tries < (1 << 20); ++tries) {
              const uint64_t ds = sys_relaxed(&ctl->desc[s].seq);
              if (ds != kDescWriting && ds < later) {
                __builtin_amdgcn_s_sleep(2);
                continue;
              }
              held = desc_ntiles(&ctl->desc[s], later, lnt);
              if (held || ds != later) break;
            }
            if (!held && sys_relaxed(&ctl->desc[s].seq) < later) {
              // never seen: report it to the host, which stops serving with an error
              __hip_atomic_store(&ctl->fault, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
              if (open_count) report();
              leave = true;
              break;
            }
            nt_seq = held ? later : ~0ull;
            ntiles = held ? lnt : 0;
            if (held && (int64_t)wc < lnt) { got_seq = (int64_t)later; got_tile = (int64_t)wc; }
            else moved_on = true;
            break;
          }
          if (got_seq >= 0 || leave) break;
          if (moved_on) {
            if (open_count && cur_seq == seq) report();  // leaving request seq
            ++seq;
            if (fin_seq >= 0) break;
          }
        } else {
          if (sys_relaxed(&ctl->stop)) {
            leave = true;
            break;
          }
          if (__builtin_amdgcn_s_memrealtime() - idle_since > idle_ticks) {
            // idle: end the launch for every workgroup
            __hip_atomic_store(&dev->drain, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (open_count) report();  // (none expected: every published request has been left)
            leave = true;
            break;
          }
          // idle: back off up to ~4 us between polls of host memory
          for (int i = 0; i < backoff; ++i) __builtin_amdgcn_s_sleep(16);
          backoff = backoff < 8 ? 2 * backoff : 8;
        }
      }
      backoff = 1;
      // -1: exit (after finalizing, if fin_seq is set), -2: nothing claimed but a request to finalize
      claim_info[0] = got_seq >= 0 ? got_seq : (fin_seq >= 0 && !leave ? -2 : -1);
      claim_info[1] = got_tile;
      claim_info[2] = fin_seq;
      if (got_seq >= 0 && (uint64_t)got_seq != cur_seq) {
        const ServeDesc* d = &ctl->desc[got_seq % slots];
        cur.knots = sys_relaxed(&d->knots);
        cur.points = sys_relaxed(&d->points);
        cur.K = sys_relaxed(&d->K);
        cur.Np = sys_relaxed(&d->Np);
        cur.nblk = sys_relaxed(&d->nblk);
        cur.ntiles = sys_relaxed(&d->ntiles);
        cur.done_target = sys_relaxed(&d->done_target);
        cur.d = sys_relaxed(&d->d);
        cur.J = sys_relaxed(&d->J);
        cur.minkey = sys_relaxed(&d->minkey);
        cur.dmin = sys_relaxed(&d->dmin);
        cur.argmin = sys_relaxed(&d->argmin);
        cur.Jmin = sys_relaxed(&d->Jmin);
        cur.want_grad = sys_relaxed(&d->want_grad);
        cur.seq = (uint64_t)got_seq;
        cur_seq = (uint64_t)got_seq;
      }
      if (got_seq >= 0) ++open_count;
    }
    __syncthreads();
    const int64_t gs = claim_info[0];
    if (claim_info[2] >= 0) {
      // this workgroup completed request fin.seq: per-knot minimum, key scratch restored
      if (fin.dmin) {
        for (int64_t k = tid; k < fin.K; k += Geo<W, MODE>::THREADS) {
          const unsigned long long key = __hip_atomic_load(fin.minkey + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const uint32_t o = (uint32_t)(key >> 32);
          const uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
          fin.dmin[k] = __uint_as_float(u);
          fin.argmin[k] = key == ~0ull ? 0 : (int32_t)(uint32_t)(key & 0xffffffffu);
          fin.minkey[k] = ~0ull;
        }
      }
      if (fin.Jmin) {
        // J at the argmin pairs (knot k, point argmin[k]): the pair-list tiles of
        // gcdf_query's Jmin pass, run by this workgroup
        __threadfence();
        __syncthreads();  // every argmin written above is visible to the workgroup
        Job pj{};
        pj.knots = fin.knots;
        pj.points = fin.points;
        pj.K = fin.K;
        pj.Np = fin.Np;
        pj.pidx32 = fin.argmin;
        pj.npairs = fin.K;
        pj.J = fin.Jmin;
        for (int64_t q0 = 0; q0 < fin.K; q0 += kTileQ)
          process_tile<W, MODE, true, false, false, SPH>(net, pj, 1, 0, q0, tc);
      }
      __threadfence_system();
      __syncthreads();
      if (tid == 0)
        __hip_atomic_store(&ctl->complete[fin.seq % slots], fin.seq + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    if (gs == -1) break;
    if (gs < 0) continue;
    const int64_t t = claim_info[1];
    Job job{};
    job.knots = cur.knots;
    job.points = cur.points;
    job.K = cur.K;
    job.Np = cur.Np;
    job.d = cur.d;
    job.J = cur.J;
    job.minkey = cur.minkey;
    const int64_t kk = t / cur.nblk;
    process_tile<W, MODE, false, false, false, SPH>(net, job, cur.want_grad, kk, (t - kk * cur.nblk) * kTileQ, tc);
    if (tid == 0) idle_since = __builtin_amdgcn_s_memrealtime();
  }
  report_overflow<W, MODE>(net, tc);
}

template <int W, int MODE, bool SPH>
static hipError_t launch_serve_t(const DevNet& net, ServeCtl* ctl, ServeDev* dev, uint64_t first_seq,
                                 uint64_t idle_ticks, uint32_t epoch, int num_cu, hipStream_t s) {
  hipLaunchKernelGGL((serve_loop<W, MODE, SPH>), dim3(num_cu), dim3((Geo<W, MODE>::THREADS)), 0, s, net, ctl, dev, first_seq, idle_ticks,
                     epoch);
  return hipGetLastError();
}

template <bool SPH>
static hipError_t launch_serve_k(const DevNet& net, ServeCtl* ctl, ServeDev* dev, uint64_t first_seq,
                                 uint64_t idle_ticks, uint32_t epoch, int num_cu, hipStream_t s) {
  if (net.width == 256) {
    switch (net.mode) {
      case kFP32: return launch_serve_t<256, kFP32, SPH>(net, ctl, dev, first_seq, idle_ticks, epoch, num_cu, s);
      case kBF16: return launch_serve_t<256, kBF16, SPH>(net, ctl, dev, first_seq, idle_ticks, epoch, num_cu, s);
      case kBF16X2F16: return launch_serve_t<256, kBF16X2F16, SPH>(net, ctl, dev, first_seq, idle_ticks, epoch, num_cu, s);
      default: return launch_serve_t<256, kBF16X2, SPH>(net, ctl, dev, first_seq, idle_ticks, epoch, num_cu, s);
    }
  }
  switch (net.mode) {
    case kFP32: return launch_serve_t<512, kFP32, SPH>(net, ctl, dev, first_seq, idle_ticks, epoch, num_cu, s);
    case kBF16: return launch_serve_t<512, kBF16, SPH>(net, ctl, dev, first_seq, idle_ticks, epoch, num_cu, s);
    case kBF16X2F16: return launch_serve_t<512, kBF16X2F16, SPH>(net, ctl, dev, first_seq, idle_ticks, epoch, num_cu, s);
    default: return launch_serve_t<512, kBF16X2, SPH>(net, ctl, dev, first_seq, idle_ticks, epoch, num_cu, s);
  }
}

hipError_t launch_serve(const DevNet& net, ServeCtl* ctl, ServeDev* dev, uint64_t first_seq, uint64_t idle_ticks,
                        uint32_t epoch, int num_cu, hipStream_t s) {
  return net.in_dim == kInDimSphere ? launch_serve_k<true>(net, ctl, dev, first_seq, idle_ticks, epoch, num_cu, s)
                                    : launch_serve_k<false>(net, ctl, dev, first_seq, idle_ticks, epoch, num_cu, s);
}


}  // namespace gcdf
