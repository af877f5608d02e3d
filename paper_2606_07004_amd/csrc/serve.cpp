// Serving scheduler (continuous batching).  See serve.h.
#include "serve.h"

#include <algorithm>
#include <chrono>

ld_ctx::ld_ctx() = default;
ld_ctx::~ld_ctx() = default;

namespace ld {

Server::Server(ld_ctx* ctx) : ctx_(ctx) {
  budget_ = (size_t)ctx->opts.hbm_budget_bytes;
  slots_.resize((size_t)ctx->opts.max_slots);
  thread_ = std::thread([this] { loop(); });
}

Server::~Server() {
  {
    std::unique_lock<std::mutex> lk(mu_);
    stop_ = true;
  }
  cv_work_.notify_all();
  if (thread_.joinable()) thread_.join();
  (void)hipSetDevice(ctx_->device);
  if (stream_) {
    (void)hipStreamSynchronize(stream_);
    (void)hipStreamDestroy(stream_);
  }
  for (Slot& s : slots_) {
    if (s.done_ev) (void)hipEventDestroy(s.done_ev);
    if (s.hpack) (void)hipHostFree(s.hpack);
    if (s.mem) (void)hipFree(s.mem);
  }
}

ld_status Server::submit(ld_matrix* a, const ld_params& p, uint64_t* ticket) {
  std::unique_ptr<Request> rq(new Request());
  rq->run.reset(new Run(a, p));
  rq->run->set_submit_time(now_seconds());
  ld_status rc = rq->run->validate();
  if (rc != LD_OK) return rc;
  rq->bytes = rq->run->device_bytes();
  if (rq->bytes > budget_)
    return set_error(LD_E_NO_MEMORY, "request needs " + std::to_string(rq->bytes) +
                                         " device bytes, more than the whole serving budget");
  a->inflight.fetch_add(1);
  std::unique_lock<std::mutex> lk(mu_);
  rq->ticket = next_ticket_++;
  *ticket = rq->ticket;
  live_[rq->ticket] = true;
  queue_.push_back(std::move(rq));
  ++stats_.submitted;
  lk.unlock();
  cv_work_.notify_all();
  return LD_OK;
}

ld_status Server::poll(uint64_t ticket, ld_result* out, bool wait) {
  std::unique_lock<std::mutex> lk(mu_);
  if (!live_.count(ticket)) return set_error(LD_E_UNKNOWN_TICKET, "unknown or retired ticket");
  for (;;) {
    auto it = done_.find(ticket);
    if (it != done_.end()) {
      Done d = it->second;
      done_.erase(it);
      live_.erase(ticket);
      lk.unlock();
      if (d.status != LD_OK) return set_error(d.status, d.error);
      *out = d.result;
      return LD_OK;
    }
    if (!wait) return LD_PENDING;
    cv_done_.wait(lk);
  }
}

Server::Stats Server::stats() {
  std::unique_lock<std::mutex> lk(mu_);
  Stats st = stats_;
  st.held_bytes = held_;
  st.budget_bytes = budget_;
  return st;
}

void Server::finish(Slot& s, ld_status st, const ld_result* res, const std::string& err) {
  Done d;
  d.status = st;
  if (res) d.result = *res;
  d.error = err;
  ld_matrix* a = s.req->run->matrix();
  {
    std::unique_lock<std::mutex> lk(mu_);
    done_[s.req->ticket] = d;
    ++stats_.completed;
  }
  a->inflight.fetch_sub(1);
  s.req.reset();
  s.enqueued_all = false;
  s.bound = false;
  cv_done_.notify_all();
}

void Server::loop() {
  (void)hipSetDevice(ctx_->device);
  for (;;) {
    // admission: FIFO, skipping ahead over requests that do not fit yet
    {
      std::unique_lock<std::mutex> lk(mu_);
      bool any_active = false;
      for (Slot& s : slots_) any_active = any_active || (bool)s.req;
      if (!any_active && queue_.empty()) {
        if (stop_) return;
        cv_work_.wait(lk, [&] { return stop_ || !queue_.empty(); });
        if (stop_ && queue_.empty()) return;
      }
      // each admitted request takes the free slot with the smallest buffer
      // that already fits it (no new memory), else the free slot with the
      // largest buffer, grown to the request's size.  The ledger charges
      // every slot's buffer, idle ones included: a growth that would take the
      // buffers past the budget first releases idle buffers of other slots
      // (largest first), and the request waits when even that is not enough
      for (auto it = queue_.begin(); it != queue_.end();) {
        const size_t want = (*it)->bytes;
        Slot* fit = nullptr;
        Slot* big = nullptr;
        for (Slot& s : slots_) {
          // a slot whose buffer is being given up takes no request this tick
          if (s.req || s.release) continue;
          if (s.mem_bytes >= want && (!fit || s.mem_bytes < fit->mem_bytes)) fit = &s;
          if (!big || s.mem_bytes > big->mem_bytes) big = &s;
        }
        Slot* s = fit ? fit : big;
        if (!s) break;  // no free slot
        if (!fit) {
          // growth: the slot's buffer goes from its size to `want`
          const size_t have = s->mem_bytes;
          size_t need = held_ - have + want;
          if (need > budget_) {
            std::vector<Slot*> idle;
            for (Slot& o : slots_)
              if (&o != s && !o.req && !o.release && o.mem_bytes > 0) idle.push_back(&o);
            std::sort(idle.begin(), idle.end(),
                      [](const Slot* a, const Slot* b) { return a->mem_bytes > b->mem_bytes; });
            size_t freeable = 0;
            for (Slot* o : idle) freeable += o->mem_bytes;
            if (need - std::min(need, freeable) > budget_) {
              ++it;  // waits for running requests to finish
              continue;
            }
            for (Slot* o : idle) {
              if (need <= budget_) break;
              o->release = true;
              held_ -= o->mem_bytes;
              need -= o->mem_bytes;
            }
          }
          held_ = held_ - have + want;
          s->want_bytes = want;
        } else {
          s->want_bytes = s->mem_bytes;
        }
        s->req = std::move(*it);
        it = queue_.erase(it);
      }
      int act = 0;
      for (Slot& s : slots_) act += s.req ? 1 : 0;
      if (act > stats_.peak_active) stats_.peak_active = act;
      if (held_ > stats_.peak_bytes) stats_.peak_bytes = held_;
      stats_.held_bytes = held_;
      ++stats_.ticks;
    }
    // bind newly admitted requests
    if (!stream_ && hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking) != hipSuccess) {
      stream_ = nullptr;
      for (Slot& s : slots_)
        if (s.req) finish(s, LD_E_DEVICE, nullptr, "stream creation failed");
      continue;
    }
    // idle buffers given up to make room (their requests finished: the
    // stream is drained first, as freeing device memory synchronises anyway)
    bool synced = false;
    for (Slot& s : slots_) {
      if (!s.release) continue;
      if (!synced) {
        (void)hipStreamSynchronize(stream_);
        synced = true;
      }
      if (s.mem) (void)hipFree(s.mem);
      s.mem = nullptr;
      s.mem_bytes = 0;
      s.release = false;
      ++stats_.buffer_frees;
    }
    for (Slot& s : slots_) {
      if (!s.req || s.enqueued_all || s.bound) continue;
      if (!s.done_ev && hipEventCreateWithFlags(&s.done_ev, hipEventDisableTiming) != hipSuccess) {
        s.done_ev = nullptr;
        finish(s, LD_E_DEVICE, nullptr, "event creation failed");
        continue;
      }
      if (!s.hpack && hipHostMalloc(&s.hpack, kHostPackBytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        s.hpack = nullptr;
        finish(s, LD_E_DEVICE, nullptr, "pinned result buffer allocation failed");
        continue;
      }
      if (s.mem_bytes < s.want_bytes) {
        if (s.mem) {
          (void)hipStreamSynchronize(stream_);
          (void)hipFree(s.mem);
          s.mem = nullptr;
          ++stats_.buffer_frees;
        }
        s.mem_bytes = 0;
        if (hipMalloc(&s.mem, s.want_bytes) != hipSuccess) {
          (void)hipGetLastError();
          s.mem = nullptr;
          {
            std::unique_lock<std::mutex> lk(mu_);
            held_ -= s.want_bytes;  // charged at admission, never allocated
          }
          finish(s, LD_E_NO_MEMORY, nullptr, "device allocation for a request failed");
          continue;
        }
        s.mem_bytes = s.want_bytes;
        ++stats_.buffer_allocs;
      }
      // a slot's memory is reused only after its previous request's work:
      // every request runs on the one scheduler stream, in order
      s.req->run->set_host_pack(s.hpack);
      ld_status brc = s.req->run->bind(s.mem, s.mem_bytes);
      if (brc != LD_OK) {
        finish(s, brc, nullptr, ld_last_error());
        continue;
      }
      s.bound = true;
    }
    // steps_per_tick rounds: in each, every resident request advances by one
    // stage (its own launches) or by one Krylov step; the Krylov steps of a
    // round go to the device together, one launch per kernel for all of them
    for (int rep = 0; rep < steps_per_tick_; ++rep) {
      std::vector<StepPlan> plans;
      std::vector<Slot*> owners;
      for (Slot& s : slots_) {
        if (!s.req || s.enqueued_all || !s.bound) continue;
        bool done = false, planned = false;
        StepPlan pl;
        const ld_status rc = s.req->run->advance(stream_, 1, &done, &pl, &planned);
        if (rc != LD_OK) {
          (void)hipStreamSynchronize(stream_);
          finish(s, rc, nullptr, ld_last_error());
          continue;
        }
        if (planned) {
          plans.push_back(pl);
          owners.push_back(&s);
        }
        if (done) {
          s.enqueued_all = true;
          (void)hipEventRecord(s.done_ev, stream_);
        }
      }
      if (!plans.empty()) {
        const hipError_t e = launch_step_plans(stream_, plans);
        if (e != hipSuccess) {
          (void)hipStreamSynchronize(stream_);
          for (Slot* o : owners)
            if (o->req) finish(*o, LD_E_DEVICE, nullptr, hipGetErrorString(e));
        }
        stats_.batched_steps += plans.size();
        ++stats_.batched_launches;
      }
    }
    // retire finished requests
    bool pending = false;
    for (Slot& s : slots_) {
      if (!s.req || !s.enqueued_all) continue;
      const hipError_t q = hipEventQuery(s.done_ev);
      if (q == hipErrorNotReady) {
        pending = true;
        continue;
      }
      ld_result res{};
      ld_status rc = (q == hipSuccess) ? s.req->run->collect(stream_, &res, nullptr, s.done_ev)
                                       : set_error(LD_E_DEVICE, hipGetErrorString(q));
      finish(s, rc, rc == LD_OK ? &res : nullptr, rc == LD_OK ? std::string() : ld_last_error());
    }
    bool all_enqueued = true;
    for (Slot& s : slots_)
      if (s.req && !s.enqueued_all) all_enqueued = false;
    // everything resident is enqueued and still running: back off briefly
    if (pending && all_enqueued) std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
}

}  // namespace ld
