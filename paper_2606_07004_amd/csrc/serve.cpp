// Serving scheduler (continuous batching).  See serve.h.
#include "serve.h"

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
  for (Slot& s : slots_) {
    if (s.stream) {
      (void)hipStreamSynchronize(s.stream);
      (void)hipStreamDestroy(s.stream);
    }
    if (s.done_ev) (void)hipEventDestroy(s.done_ev);
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
  return stats_;
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
    used_ -= s.req->bytes;
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
      for (Slot& s : slots_) {
        if (s.req || queue_.empty()) continue;
        for (auto it = queue_.begin(); it != queue_.end(); ++it) {
          if (used_ + (*it)->bytes <= budget_) {
            s.req = std::move(*it);
            queue_.erase(it);
            used_ += s.req->bytes;
            break;
          }
        }
      }
      int act = 0;
      for (Slot& s : slots_) act += s.req ? 1 : 0;
      if (act > stats_.peak_active) stats_.peak_active = act;
      if (used_ > stats_.peak_bytes) stats_.peak_bytes = used_;
      ++stats_.ticks;
    }
    // bind newly admitted requests and enqueue a slice of every resident one
    for (Slot& s : slots_) {
      if (!s.req || s.enqueued_all) continue;
      if (!s.stream) {
        if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s.done_ev, hipEventDisableTiming) != hipSuccess) {
          finish(s, LD_E_DEVICE, nullptr, "stream creation failed");
          continue;
        }
      }
      if (!s.bound) {
        if (s.mem_bytes < s.req->bytes) {
          if (s.mem) {
            (void)hipStreamSynchronize(s.stream);
            (void)hipFree(s.mem);
            s.mem = nullptr;
            s.mem_bytes = 0;
          }
          if (hipMalloc(&s.mem, s.req->bytes) != hipSuccess) {
            s.mem = nullptr;
            finish(s, LD_E_NO_MEMORY, nullptr, "device allocation for a request failed");
            continue;
          }
          s.mem_bytes = s.req->bytes;
        }
        ld_status brc = s.req->run->bind(s.mem, s.mem_bytes);
        if (brc != LD_OK) {
          finish(s, brc, nullptr, ld_last_error());
          continue;
        }
        s.bound = true;
      }
      bool done = false;
      ld_status rc = s.req->run->advance(s.stream, steps_per_tick_, &done);
      if (rc != LD_OK) {
        (void)hipStreamSynchronize(s.stream);
        finish(s, rc, nullptr, ld_last_error());
        continue;
      }
      if (done) {
        s.enqueued_all = true;
        (void)hipEventRecord(s.done_ev, s.stream);
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
      ld_status rc = (q == hipSuccess) ? s.req->run->collect(s.stream, &res, nullptr)
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
