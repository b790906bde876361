// Host loop of the iterative solves (the Section 4 program repeated until the
// change between iterates is small enough): iterations are queued on the
// stream, and each checked iteration's scalars are copied into pinned host
// memory behind it. The loop queues the iteration after a check before it
// waits for that check, so the GPU does not idle while the host reads the
// scalars back and decides. An iteration alternates between the two buffers
// of each pair, so the one queued ahead only reads the checked iterate and
// writes the other buffer: when the check ends the loop (or switches the
// precision) the loop rolls back to the checked iterate, and the results are
// those of a loop that waited at every check.
//
// A check is not run ahead when the residual read back before it, shrunk by
// the last observed ratio between checks, predicts that it may end the loop
// (or switch the precision): running ahead then would likely cost a whole
// iteration to save one round trip.
#pragma once

#include <math.h>

#include <mutex>
#include <vector>

#include "common.h"

namespace cagra {

// Pinned host slots and events through which a solve reads its check values
// back. Created per device on first use, kept until the process ends, and lent
// to one solve at a time (concurrent solves take distinct ones).
constexpr size_t kReadbackBytes = CAGRA_PPR_COLS * 4 * sizeof(double);  // the largest set read back at once

struct Readback {
    int dev = -1;
    unsigned char *host = nullptr;  // two slots of kReadbackBytes
    hipEvent_t ev[2] = {nullptr, nullptr};
};

inline std::mutex &readback_mutex() {
    static std::mutex mu;
    return mu;
}
inline std::vector<Readback *> &readback_free_list() {
    static std::vector<Readback *> v;
    return v;
}

class ReadbackLease {
  public:
    ReadbackLease() = default;
    ReadbackLease(const ReadbackLease &) = delete;
    ReadbackLease &operator=(const ReadbackLease &) = delete;
    ~ReadbackLease() {
        if (!rb_) return;
        std::lock_guard<std::mutex> lock(readback_mutex());
        readback_free_list().push_back(rb_);
    }
    cagra_status acquire() {
        int dev = 0;
        CAGRA_HIP_CHECK(hipGetDevice(&dev));
        {
            std::lock_guard<std::mutex> lock(readback_mutex());
            auto &fl = readback_free_list();
            for (size_t i = 0; i < fl.size(); ++i)
                if (fl[i]->dev == dev) {
                    rb_ = fl[i];
                    fl.erase(fl.begin() + (long)i);
                    return CAGRA_OK;
                }
        }
        Readback *r = new Readback;
        r->dev = dev;
        hipError_t e = hipHostMalloc((void **)&r->host, 2 * kReadbackBytes, hipHostMallocDefault);
        for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&r->ev[i], hipEventDisableTiming);
        if (e != hipSuccess) {
            for (int i = 0; i < 2; ++i)
                if (r->ev[i]) (void)hipEventDestroy(r->ev[i]);
            if (r->host) (void)hipHostFree(r->host);
            delete r;
            return fail(CAGRA_E_HIP, "pinned read-back buffer: %s", hipGetErrorString(e));
        }
        rb_ = r;
        return CAGRA_OK;
    }
    Readback *get() const { return rb_; }

  private:
    Readback *rb_ = nullptr;
};

enum class CheckOutcome { kContinue, kConverged, kSwitch, kError };

// The residual expected at the next check: the last one read back times the
// last ratio between consecutive checks (at most 1); infinite before any.
inline double predict_residual(double r_last, double r_prev) {
    if (!(isfinite(r_last) && isfinite(r_prev) && r_prev > 0.0)) return r_last;
    return r_last * fmin(r_last / r_prev, 1.0);
}

// Runs a solve whose per-problem parts Ops supplies:
//   State state() const / void restore(const State&)  the loop position
//       (current buffer, iteration counts in State::iters, precision) to roll
//       back to;
//   int32_t iters() const                              iterations queued;
//   cagra_status step()                                queues one iteration;
//   const void *dev_check() const, size_t check_bytes() const
//                                                      the device values to read
//                                                      back after the current
//                                                      iterate (<= kReadbackBytes);
//   CheckOutcome decide(const State &at, const void *h, double *residual,
//                 cagra_status *err)                   decides from the values h
//                                                      read back at position at
//                                                      (kError sets *err);
//   bool may_end(double predicted) const               whether a check with this
//                                                      residual may end or switch;
//   cagra_status switch_precision()                    applies kSwitch at the
//                                                      restored position.
// Returns CAGRA_OK when a check converged, CAGRA_E_NOT_CONVERGED when the
// check after max_iters iterations did not, or the first error; the position
// of Ops is that of the last check read back. The stream is synchronized
// before the return, so no queued iteration writes after it.
template <class Ops>
cagra_status pipelined_solve(Ops &ops, int32_t max_iters, int32_t check_every, hipStream_t st) {
    using State = decltype(ops.state());
    struct Check {
        State at;
        int slot;
    };
    ReadbackLease lease;
    cagra_status s = lease.acquire();
    if (s != CAGRA_OK) return s;
    Readback *rb = lease.get();
    Check q[2] = {};
    int nq = 0, slot = 0;
    double r_last = INFINITY, r_prev = INFINITY;
    cagra_status err = CAGRA_OK;
    bool converged = false;
    auto is_check = [&](int32_t i) { return i % check_every == 0 || i >= max_iters; };
    // queues one iteration, and the copy of its scalars when it is a check
    auto advance = [&]() -> cagra_status {
        cagra_status t = ops.step();
        if (t != CAGRA_OK) return t;
        if (!is_check(ops.iters())) return CAGRA_OK;
        unsigned char *dst = rb->host + (size_t)slot * kReadbackBytes;
        CAGRA_HIP_CHECK(hipMemcpyAsync(dst, ops.dev_check(), ops.check_bytes(), hipMemcpyDeviceToHost, st));
        CAGRA_HIP_CHECK(hipEventRecord(rb->ev[slot], st));
        q[nq++] = Check{ops.state(), slot};
        slot ^= 1;
        return CAGRA_OK;
    };
    for (;;) {
        while (nq == 0) {  // up to the next check (the cap is always one)
            if ((err = advance()) != CAGRA_OK) break;
        }
        if (err != CAGRA_OK) break;
        if (nq == 1 && ops.iters() < max_iters && !ops.may_end(predict_residual(r_last, r_prev))) {
            if ((err = advance()) != CAGRA_OK) break;
        }
        const hipError_t e = hipEventSynchronize(rb->ev[q[0].slot]);
        if (e != hipSuccess) {
            err = fail(CAGRA_E_HIP, "hipEventSynchronize: %s", hipGetErrorString(e));
            break;
        }
        double resid = INFINITY;
        const CheckOutcome v = ops.decide(q[0].at, rb->host + (size_t)q[0].slot * kReadbackBytes, &resid, &err);
        r_prev = r_last;
        r_last = resid;
        if (v == CheckOutcome::kContinue) {
            if (q[0].at.iters >= max_iters) break;  // the cap's check (nothing is queued after it)
            if (nq == 2) q[0] = q[1];
            --nq;
            continue;
        }
        ops.restore(q[0].at);  // back to the checked iterate; anything queued after it is dropped
        nq = 0;
        if (v == CheckOutcome::kConverged) {
            converged = true;
            break;
        }
        if (v == CheckOutcome::kError) break;
        if ((err = ops.switch_precision()) != CAGRA_OK) break;
        if (ops.iters() >= max_iters) break;  // switched at the cap's check
    }
    const hipError_t e = hipStreamSynchronize(st);
    if (err != CAGRA_OK) return err;
    if (e != hipSuccess) return fail(CAGRA_E_HIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    return converged ? CAGRA_OK : CAGRA_E_NOT_CONVERGED;
}

}  // namespace cagra
