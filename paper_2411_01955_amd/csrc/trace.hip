// Per-kernel duration tracing with HIP events.
//
// When enabled, every launch site brackets its kernel with two events
// recorded on the kernel's own stream (without the system-scope release
// fence a default event performs, so an interval holds the kernel and its
// dispatch only); pnp_trace_read() waits for the
// recorded events and reports, per kernel name, the launch count and the
// summed duration.  Disabled (the default), a launch site costs one branch.
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "trace.hpp"

namespace pnp {

namespace {

struct Pending {
  const char* name;
  hipEvent_t a, b;
};

struct TraceState {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<Pending> pending;
  std::map<std::string, std::pair<long long, double>> acc;  // name -> (count, ms)
};

TraceState& state() {
  static TraceState* s = new TraceState();  // leaked on purpose: outlives static destructors
  return *s;
}

hipEvent_t take_event(TraceState& s) {
  if (!s.pool.empty()) {
    hipEvent_t e = s.pool.back();
    s.pool.pop_back();
    return e;
  }
  // no system-scope fence when the event completes: the events only time,
  // and the fence's cache writeback and invalidation would be counted in
  // the kernel's interval and slow the kernel after it
  hipEvent_t e;
  PNP_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  return e;
}

void drain(TraceState& s) {
  for (auto& p : s.pending) {
    PNP_HIP(hipEventSynchronize(p.b));
    float ms = 0.f;
    PNP_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    auto& slot = s.acc[p.name];
    slot.first += 1;
    slot.second += ms;
    s.pool.push_back(p.a);
    s.pool.push_back(p.b);
  }
  s.pending.clear();
}

}  // namespace

bool trace_on() { return state().on; }

TraceScope::TraceScope(hipStream_t s, const char* name) : stream_(s), name_(name), active_(false) {
  TraceState& st = state();
  if (!st.on) return;
  std::lock_guard<std::mutex> g(st.mu);
  if (st.pending.size() > 65536) drain(st);
  a_ = take_event(st);
  b_ = take_event(st);
  PNP_HIP(hipEventRecord(a_, stream_));
  active_ = true;
}

TraceScope::~TraceScope() {
  if (!active_) return;
  TraceState& st = state();
  std::lock_guard<std::mutex> g(st.mu);
  if (hipEventRecord(b_, stream_) == hipSuccess) {
    st.pending.push_back({name_, a_, b_});
  } else {
    st.pool.push_back(a_);
    st.pool.push_back(b_);
  }
}

void trace_enable(bool on) {
  TraceState& st = state();
  std::lock_guard<std::mutex> g(st.mu);
  st.on = on;
}

std::string trace_read_json() {
  TraceState& st = state();
  std::lock_guard<std::mutex> g(st.mu);
  drain(st);
  std::string out = "{";
  bool first = true;
  for (auto& kv : st.acc) {
    char buf[256];
    snprintf(buf, sizeof(buf), "%s\"%s\": [%lld, %.6f]", first ? "" : ", ", kv.first.c_str(),
             kv.second.first, kv.second.second);
    out += buf;
    first = false;
  }
  out += "}";
  st.acc.clear();
  return out;
}

}  // namespace pnp
