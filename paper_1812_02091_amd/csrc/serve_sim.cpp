// Host-only run of the serving admission policy (admission.h) against a fake
// executor on a virtual clock: the same Admission class the serving worker
// uses, with each launch lasting t_fixed + t_per_query x (queries in it).
// Declared in include/lcemd.h (lcemd_serve_sim); needs no GPU.
#include <algorithm>
#include <cstdint>
#include <queue>
#include <vector>

#include "../../include/lcemd.h"
#include "admission.h"

namespace {
struct SimQ {
  int id;
  int words;
};
}  // namespace

extern "C" int lcemd_serve_sim(int32_t nq, const double* arrival_s, const int32_t* words, int32_t lanes,
                               int32_t max_slots, int32_t max_words, int64_t budget, double per_query_bytes,
                               double t_fixed_s, double t_per_query_s, int32_t* status, int32_t* lane,
                               int32_t* launch, double* start_s, double* finish_s) {
  if (nq < 0 || !arrival_s || !words || lanes < 1 || max_words < 1 || !status || !lane || !launch || !start_s ||
      !finish_s)
    return LCEMD_E_INVALID_ARG;
  for (int i = 1; i < nq; ++i)
    if (arrival_s[i] < arrival_s[i - 1]) return LCEMD_E_INVALID_ARG;
  const int slots = lcemd_serve::plan_slots(budget, per_query_bytes, 0.0, lanes, max_slots);
  if (slots < 1) return LCEMD_E_CAPACITY;
  lcemd_serve::Admission<SimQ> adm(lanes, slots, max_words);
  // completions: (time, lane, launch id)
  using Ev = std::pair<double, std::pair<int, int>>;
  std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> running;
  std::vector<std::vector<int>> members;
  int next_arrival = 0, launches = 0;
  double now = 0.0;
  std::vector<SimQ> batch;
  while (next_arrival < nq || !running.empty() || adm.waiting() > 0) {
    // the next event: a completion or an arrival, whichever comes first
    const double ta = next_arrival < nq ? arrival_s[next_arrival] : 1e300;
    const double tc = running.empty() ? 1e300 : running.top().first;
    now = std::min(ta, tc);
    while (!running.empty() && running.top().first <= now) {
      const int l = running.top().second.first, id = running.top().second.second;
      running.pop();
      for (int q : members[id]) finish_s[q] = now;
      adm.done(l);
    }
    while (next_arrival < nq && arrival_s[next_arrival] <= now) {
      const int q = next_arrival++;
      if (!adm.fits(words[q])) {  // longer than a lane's words: refused at submission
        status[q] = LCEMD_E_CAPACITY;
        lane[q] = launch[q] = -1;
        start_s[q] = finish_s[q] = arrival_s[q];
        continue;
      }
      status[q] = LCEMD_OK;
      adm.push(SimQ{q, words[q]});
    }
    int l;
    while ((l = adm.next(batch)) >= 0) {
      members.emplace_back();
      for (const SimQ& s : batch) {
        lane[s.id] = l;
        launch[s.id] = launches;
        start_s[s.id] = now;
        members.back().push_back(s.id);
      }
      running.push({now + t_fixed_s + t_per_query_s * (double)batch.size(), {l, launches}});
      ++launches;
    }
    if (next_arrival >= nq && running.empty() && adm.waiting() > 0) return LCEMD_E_CAPACITY;  // cannot happen
  }
  return slots;
}
