// Serving loop: extrapolation jobs of different sizes are admitted by their
// HBM footprint into a caller-owned device arena, stay resident while they
// run, and every step advances all resident jobs by one layer in shared
// persistent launches (continuous batching: a job that arrives while others
// are on the GPU joins the next launch once memory and a slot are free).
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "nze.h"
#include "nze_internal.h"

using nze::fail;

namespace {

struct Job {
  int64_t id = 0;
  mpo_config cfg{};
  std::vector<int32_t> layer_gates;   // gates per layer
  std::vector<int32_t> layer_off;     // offset of each layer's left sites
  std::vector<int32_t> left_sites;
  std::vector<size_t> ptm_off;        // offset (doubles) of each layer's PTMs
  std::vector<double> ptm;
  int32_t n_obs = 0;
  std::vector<uint8_t> paulis;
  // run state
  int state = 0;                      // 0 queued, 1 resident, 2 done, <0 error
  int passed = 0;                     // steps in which a later job was admitted first
  int layer = 0;
  mpo_t* h = nullptr;
  size_t off = 0, bytes = 0;          // arena block
  double t_submit = 0, t_admit = 0, t_done = 0;
  std::vector<double> values, fidelity;
};

}  // namespace

// steps in which a queued job may be passed by later jobs that fit
constexpr int BACKFILL_STEPS = 16;

struct nze_server {
  char* arena = nullptr;
  size_t arena_bytes = 0;
  int max_active = 0;
  void* stream = nullptr;
  int64_t next_id = 1;
  std::deque<Job*> queue;
  std::vector<Job*> active;
  std::map<int64_t, Job*> jobs;
  std::map<size_t, size_t> used;      // arena offset -> bytes
  size_t high_water = 0;
  int64_t launches = 0;
  std::chrono::steady_clock::time_point t0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  // first fit, 256-byte aligned
  bool alloc(size_t bytes, size_t* off) {
    size_t cur = 0;
    for (const auto& kv : used) {
      if (kv.first >= cur + bytes) break;
      cur = std::max(cur, (kv.first + kv.second + 255) & ~(size_t)255);
    }
    if (cur + bytes > arena_bytes) return false;
    used[cur] = bytes;
    *off = cur;
    size_t top = 0;
    for (const auto& kv : used) top = std::max(top, kv.first + kv.second);
    high_water = std::max(high_water, top);
    return true;
  }
  void release(size_t off) { used.erase(off); }
};

extern "C" int nze_server_create(nze_server_t** out, void* arena,
                                 size_t arena_bytes, int32_t max_active,
                                 void* stream) {
  if (!out || !arena || arena_bytes == 0 || max_active < 1)
    return fail(NZE_EINVAL, "bad server arguments");
  if (reinterpret_cast<uintptr_t>(arena) & 255)
    return fail(NZE_EINVAL, "arena must be 256-byte aligned");
  nze_server* s = new nze_server();
  s->arena = reinterpret_cast<char*>(arena);
  s->arena_bytes = arena_bytes;
  s->max_active = max_active;
  s->stream = stream;
  s->t0 = std::chrono::steady_clock::now();
  *out = s;
  return NZE_OK;
}

extern "C" void nze_server_free(nze_server_t* s) {
  if (!s) return;
  for (auto& kv : s->jobs) {
    if (kv.second->h) mpo_free(kv.second->h);
    delete kv.second;
  }
  delete s;
}

namespace {
constexpr int MAX_LAUNCH_MPOS = 256;   // resident workgroups of the double kernel
}  // namespace

extern "C" int nze_server_submit(nze_server_t* s, const nze_job_spec* spec,
                                 int64_t* job_id) {
  if (!s || !spec || !job_id) return fail(NZE_EINVAL, "bad submit arguments");
  mpo_config cfg{};
  cfg.n = spec->n;
  cfg.chi_max = spec->chi_max;
  cfg.n_levels = spec->n_levels;
  cfg.precision = spec->precision;
  const size_t need = mpo_footprint(&cfg);
  if (need == 0) return fail(NZE_EINVAL, "invalid job configuration");
  if (need > s->arena_bytes) return fail(NZE_ENOMEM, "job larger than the arena");
  if (spec->n_levels > MAX_LAUNCH_MPOS)
    return fail(NZE_EINVAL, "job has more levels than one layer launch holds (256)");
  if (spec->n_layers < 0 || (spec->n_layers > 0 && (!spec->layer_gates || !spec->ptm)))
    return fail(NZE_EINVAL, "bad layers");
  if (spec->n_obs < 0 || (spec->n_obs > 0 && !spec->paulis))
    return fail(NZE_EINVAL, "bad observables");
  Job* j = new Job();
  j->cfg = cfg;
  const int L = spec->n_levels;
  size_t ls_tot = 0, p_tot = 0;
  for (int t = 0; t < spec->n_layers; ++t) {
    const int g = spec->layer_gates[t];
    if (g < 0) { delete j; return fail(NZE_EINVAL, "negative gate count"); }
    j->layer_gates.push_back(g);
    j->layer_off.push_back((int32_t)ls_tot);
    j->ptm_off.push_back(p_tot);
    ls_tot += g;
    p_tot += (size_t)L * g * 256;
  }
  if (ls_tot > 0 && !spec->left_sites) { delete j; return fail(NZE_EINVAL, "no left sites"); }
  // the layers are checked here, so that a bad job is refused at submission
  // instead of failing the shared launches of the jobs resident beside it
  for (int t = 0; t < spec->n_layers; ++t) {
    const int32_t* ls = spec->left_sites + j->layer_off[t];
    for (int i = 0; i < j->layer_gates[t]; ++i) {
      if (ls[i] < 0 || ls[i] + 1 >= spec->n || (i > 0 && ls[i] - ls[i - 1] < 2)) {
        delete j;
        return fail(NZE_EINVAL, "layer sites outside the chain, unsorted or overlapping");
      }
    }
  }
  j->left_sites.assign(spec->left_sites, spec->left_sites + ls_tot);
  j->ptm.assign(spec->ptm, spec->ptm + p_tot);
  j->n_obs = spec->n_obs;
  j->paulis.assign(spec->paulis, spec->paulis + (size_t)spec->n_obs * spec->n);
  j->id = s->next_id++;
  j->t_submit = s->now();
  s->jobs[j->id] = j;
  s->queue.push_back(j);
  *job_id = j->id;
  return NZE_OK;
}

namespace {

int finish(nze_server* s, Job* j) {
  const int L = j->cfg.n_levels;
  j->values.assign((size_t)L * std::max(j->n_obs, 1), 0.0);
  j->fidelity.assign(L, 0.0);
  std::vector<double> tr(L);
  int rc = mpo_expect(j->h, j->n_obs, j->paulis.data(), j->values.data(),
                      j->fidelity.data(), tr.data());
  mpo_free(j->h);
  j->h = nullptr;
  s->release(j->off);
  j->t_done = s->now();
  j->state = rc == NZE_OK ? 2 : rc;
  // the job's inputs are no longer needed
  std::vector<double>().swap(j->ptm);
  std::vector<int32_t>().swap(j->left_sites);
  return rc;
}

}  // namespace

extern "C" int nze_server_step(nze_server_t* s, int32_t* n_active,
                               int32_t* n_queued, int32_t* n_done) {
  if (!s) return fail(NZE_EINVAL, "NULL server");
  // admission in arrival order, first fit in the arena by HBM footprint.
  // A job that does not fit yet may be passed by later ones that do
  // (backfill), in at most BACKFILL_STEPS steps; after that nothing is
  // admitted behind it until it fits, so no job waits for ever.
  {
    std::vector<Job*> waiting;          // older jobs that did not fit this step
    std::vector<Job*> keep;
    bool passed_this_step = false;
    bool closed = false;                // an old enough job blocks the rest
    for (Job* j : s->queue) {
      if (closed || (int)s->active.size() >= s->max_active) { keep.push_back(j); continue; }
      const size_t need = mpo_footprint(&j->cfg);
      size_t off;
      if (!s->alloc(need, &off)) {
        waiting.push_back(j);
        keep.push_back(j);
        if (j->passed >= BACKFILL_STEPS) closed = true;
        continue;
      }
      int rc = mpo_init(&j->h, &j->cfg, nullptr, s->arena + off, need, s->stream);
      if (rc != NZE_OK) {
        s->release(off);
        j->state = rc;
        continue;
      }
      j->off = off;
      j->bytes = need;
      j->state = 1;
      j->t_admit = s->now();
      s->active.push_back(j);
      passed_this_step = passed_this_step || !waiting.empty();
    }
    if (passed_this_step)
      for (Job* j : waiting) j->passed += 1;
    s->queue.assign(keep.begin(), keep.end());
  }
  // one layer of every resident job, batched per precision.  A job's layer
  // counter advances once its launch is enqueued; a failing launch of several
  // jobs is retried job by job, and a job whose own launch fails is ended
  // with that error (its memory released) while the others go on.
  auto launch = [&](Job* const* js, size_t k) {
    std::vector<mpo_t*> hs(k);
    std::vector<int32_t> ng(k);
    std::vector<const int32_t*> ls(k);
    std::vector<const double*> pt(k);
    for (size_t i = 0; i < k; ++i) {
      Job* j = js[i];
      hs[i] = j->h;
      ng[i] = j->layer_gates[j->layer];
      ls[i] = j->left_sites.data() + j->layer_off[j->layer];
      pt[i] = j->ptm.data() + j->ptm_off[j->layer];
    }
    const int rc = mpo_apply_layer_batch(hs.data(), (int32_t)k, ng.data(), ls.data(), pt.data());
    if (rc == NZE_OK) {
      s->launches++;
      for (size_t i = 0; i < k; ++i) js[i]->layer++;
    }
    return rc;
  };
  auto end_job = [&](Job* j, int rc) {
    mpo_free(j->h);
    j->h = nullptr;
    s->release(j->off);
    j->t_done = s->now();
    j->state = rc;
  };
  for (int prec = 0; prec < 2; ++prec) {
    std::vector<Job*> js;
    for (Job* j : s->active)
      if (j->state == 1 && j->cfg.precision == prec && j->layer < (int)j->layer_gates.size())
        js.push_back(j);
    // launches of at most MAX_LAUNCH_MPOS MPOs (levels) each, so that every
    // launch fits the co-resident grid of the persistent kernel
    size_t b = 0;
    while (b < js.size()) {
      size_t e = b;
      int mpos = 0;
      while (e < js.size()) {
        const int lv = js[e]->cfg.n_levels;
        if (e > b && mpos + lv > MAX_LAUNCH_MPOS) break;
        mpos += lv;
        ++e;
      }
      const int rc0 = launch(js.data() + b, e - b);
      if (rc0 != NZE_OK) {
        for (size_t i = b; i < e; ++i) {
          const int rc = e - b > 1 ? launch(js.data() + i, 1) : rc0;
          if (rc != NZE_OK) end_job(js[i], rc);
        }
      }
      b = e;
    }
  }
  // jobs that have run all their layers: read out and release their memory
  std::vector<Job*> keep;
  for (Job* j : s->active) {
    if (j->state != 1) continue;                 // ended by a failed launch
    if (j->layer >= (int)j->layer_gates.size()) finish(s, j);
    else keep.push_back(j);
  }
  s->active.swap(keep);
  int done = 0;
  for (auto& kv : s->jobs) done += kv.second->state == 2 ? 1 : 0;
  if (n_active) *n_active = (int32_t)s->active.size();
  if (n_queued) *n_queued = (int32_t)s->queue.size();
  if (n_done) *n_done = done;
  return NZE_OK;
}

extern "C" int nze_server_poll(nze_server_t* s, int64_t job_id, int32_t* state,
                               double* values, double* fidelity,
                               double* times) {
  if (!s) return fail(NZE_EINVAL, "NULL server");
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) return fail(NZE_EINVAL, "unknown job");
  Job* j = it->second;
  if (state) *state = j->state;
  if (j->state == 2) {
    if (values) std::memcpy(values, j->values.data(), sizeof(double) * (size_t)j->cfg.n_levels * j->n_obs);
    if (fidelity) std::memcpy(fidelity, j->fidelity.data(), sizeof(double) * j->cfg.n_levels);
  }
  if (times) { times[0] = j->t_submit; times[1] = j->t_admit; times[2] = j->t_done; }
  return NZE_OK;
}

extern "C" int nze_server_stats(nze_server_t* s, size_t* arena_high_water,
                                int64_t* launches) {
  if (!s) return fail(NZE_EINVAL, "NULL server");
  if (arena_high_water) *arena_high_water = s->high_water;
  if (launches) *launches = s->launches;
  return NZE_OK;
}
