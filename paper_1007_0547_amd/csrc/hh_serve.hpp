// Serving state of a context: worker lanes, request queue and tickets.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/hough_hier.h"
#include "hh_engine.hpp"

namespace hh {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    hh_input in{};
    int64_t pixels = 0;            // image pixels, or points of a list
    int64_t points = -1;           // edge points if known at submission (point lists, host binary images)
    int32_t depth = 0;             // finest level the request will run to
    int64_t bytes = 0;             // predicted device footprint, set when a lane admits it
    Clock::time_point t_submit, t_start, t_done;
    bool done = false;
    hh_status status = HH_OK;
    std::string error;
    hh_result* result = nullptr;
};

struct Server {
    hh_serve_config cfg{};
    std::vector<hh_ctx*> lanes;        // one context per lane, each on its own stream
    std::vector<hipStream_t> streams;
    std::vector<std::thread> workers;
    std::mutex mu;                     // queue, tickets, slab space and the stop flag
    std::condition_variable work_cv;   // a request was queued, slab space came back, or stop
    std::condition_variable done_cv;   // a request completed, or stop
    std::deque<std::shared_ptr<Request>> pending;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> tickets;   // not yet claimed by poll
    uint64_t next_ticket = 1;
    bool stop = false;
    // Device state: one slab of `budget` bytes, allocated when serving
    // starts.  The lanes' pools draw every block from it (inputs' staging,
    // level lists, cells and voters), and a result keeps its batch's blocks
    // until the last result of the batch is freed, so serving allocates no
    // device memory.  Admission by device memory: a lane takes requests
    // while their predicted footprint fits the slab's largest free interval.
    // A request's footprint is predicted as beta * E * 2^depth bytes, with E
    // its edge points (or pixels times the edge density seen so far); beta
    // and the density are running averages over completed batches (measured
    // need / sum of E * 2^depth).  The prediction sizes a batch's first
    // level arena; lists that outgrow it grow it from the level that
    // overflowed.
    char* slab = nullptr;
    SlabSpace space;
    int64_t budget = 0;
    int running = 0;                   // batches on the lanes
    int64_t slab_batches = 0, outside_batches = 0, retries = 0;
    int64_t internal_reruns = 0, internal_failures = 0;   // batches whose internal check failed, and again
    std::string first_internal_error;
    double beta = 12.0;
    double density = 0.03;
};

}  // namespace hh
