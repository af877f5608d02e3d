// Serving scheduler: continuous batching of logdet requests on one GPU.
//
// Requests wait in a FIFO until a resident slot and enough of the HBM budget
// are free; admitted requests own private device state, so a result depends
// only on its own matrix and parameters.  Each scheduler tick runs a few
// rounds; in a round every resident request advances by one stage or one
// Krylov step, and the Krylov steps of all resident requests go to the device
// as one launch per kernel (batched kernels: each request keeps the grid it
// would have alone, so its result is the same alone and in the mix).  All
// work runs on one scheduler stream; a request that finishes frees its slot
// and memory for the next one at the following tick.
#pragma once

#include "runtime.h"

namespace ld {

class Server {
 public:
  explicit Server(ld_ctx* ctx);
  ~Server();  // drains every submitted request, then stops the scheduler
  ld_status submit(ld_matrix* a, const ld_params& p, uint64_t* ticket);
  ld_status poll(uint64_t ticket, ld_result* out, bool wait);

  // scheduler statistics
  struct Stats {
    uint64_t submitted = 0, completed = 0, ticks = 0;
    uint64_t batched_steps = 0, batched_launches = 0;  // Krylov steps, batches
    size_t peak_bytes = 0;       // most device bytes the slot buffers held at once
    size_t held_bytes = 0;       // device bytes the slot buffers hold now
    uint64_t buffer_allocs = 0, buffer_frees = 0;
    size_t budget_bytes = 0;
    int peak_active = 0;
  };
  Stats stats();

 private:
  struct Request {
    uint64_t ticket = 0;
    std::unique_ptr<Run> run;
    size_t bytes = 0;
  };
  struct Slot {
    hipEvent_t done_ev = nullptr;
    void* hpack = nullptr;       // pinned buffer the request's results land in
    std::unique_ptr<Request> req;
    void* mem = nullptr;
    size_t mem_bytes = 0;        // bytes of the buffer (charged to held_)
    size_t want_bytes = 0;       // buffer size the admitted request needs
    bool release = false;        // idle buffer to free before the next binding
    bool enqueued_all = false;
    bool bound = false;
  };
  struct Done {
    ld_status status = LD_OK;
    ld_result result{};
    std::string error;
  };
  void loop();
  void finish(Slot& s, ld_status st, const ld_result* res, const std::string& err);

  ld_ctx* ctx_;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::deque<std::unique_ptr<Request>> queue_;
  std::map<uint64_t, Done> done_;
  std::map<uint64_t, bool> live_;   // submitted and not yet retired
  std::vector<Slot> slots_;
  hipStream_t stream_ = nullptr;    // the scheduler's stream
  // budget_: device bytes the slot buffers may hold; held_: what they hold
  // (idle slots keep their buffers for reuse, so they are charged too)
  size_t budget_ = 0, held_ = 0;
  uint64_t next_ticket_ = 1;
  bool stop_ = false;
  int steps_per_tick_ = 4;
  Stats stats_;
  std::thread thread_;
};

}  // namespace ld
