// Internals of the request server shared with the batch driver.
#pragma once

#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/helm_serve.h"
#include "api_common.h"

namespace helm {

double wall_ms();

struct Request {
  int64_t id = 0;
  int model = 0, n = 0;
  std::vector<long long> nodes;
  std::vector<double2> amps;
  double2* out = nullptr;
  int next_col = 0;       // next column to enter a slot
  int done_cols = 0;
  bool finished = false;
  helm_request_info info{};
};

struct Slot {
  Request* req = nullptr;
  int col = -1;
  int steps = 0;
  RefineTrack track;
};

struct Lane {
  int model = 0;
  helm_handle* h = nullptr;
  int K = 0;
  size_t bytes = 0;
  bool retire = false;          // leave the loop once idle (model removed)
  bool gone = false;            // thread joined, memory released
  std::map<int, std::unique_ptr<Method>> methods;   // by width (1, 2, 4, ..., K)
  Method& method_for(int occupied);
  DevMem F, U, R, D, nodes_d, amps_d;
  std::vector<Slot> slots;
  std::deque<Request*> queue;   // requests with columns not yet in a slot
  std::vector<long long> node_h;
  std::vector<double2> amp_h;
  std::thread th;
  int occupied() const {
    int c = 0;
    for (const Slot& s : slots) c += s.req != nullptr;
    return c;
  }
};

struct Server {
  helm_server_options opt{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  std::vector<std::unique_ptr<Lane>> lanes;
  std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
  int64_t next_id = 1;
  size_t reserved = 0;
  double t0 = 0;
  std::vector<double> lat;
  long long req_done = 0, cols_done = 0, steps = 0;
  double slot_steps = 0;
  double t_first_submit = -1, t_last_done = 0;

  void run_lane(Lane& ln);
  void finish_column(Request* r, int status, int steps, double rel, double est);
  // admit a handle (lock not held); returns the model id
  int add_model(helm_handle* h, int max_slots, int* slots_out);
  // queue n point sources (validated) for a model; returns the request
  Request* submit(int model, int n, const int64_t* nodes, const double* amps, double* u);
  // wait for the model's lane to drain, stop its thread, release its memory
  void remove_model(int model);
  void shutdown();
};

}  // namespace helm
