// Continuous-batching server for IPC time steps.
//
// Requests (a scene plus a script of per-step kinematic targets) are queued by
// taccel_server_submit.  An admission thread moves queued requests, in arrival order, into a
// new cohort as soon as their estimated device footprint fits the remaining HBM budget and
// fewer than max_cohorts cohorts are running.  A cohort is one resident Batch (all its
// scenes concatenated on the device, one launch per stage) with its own stream and host
// thread; it advances all its unfinished requests by one step per call and releases its
// memory when the last one finishes.  Cohorts admitted at different times therefore run
// concurrently on the device.  Per scene the numerics are independent of what else is in
// the batch, so a request's results do not depend on the mix it was served in.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "solver.h"

namespace tc {
namespace {

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t0, Clock::time_point t) {
  return std::chrono::duration<double, std::milli>(t - t0).count();
}

// Owned copy of a scene description.
struct OwnedScene {
  std::vector<double> verts;
  std::vector<int32_t> tets;
  std::vector<uint8_t> dirichlet;
  bool has_dirichlet = false;
  std::vector<std::vector<double>> bverts;
  std::vector<std::vector<int32_t>> btris;
  std::vector<taccel_body_desc> bodies;
  taccel_scene_desc desc{};
  int n_moving = 0;

  explicit OwnedScene(const taccel_scene_desc& d) {
    desc = d;
    verts.assign(d.soft.verts, d.soft.verts + 3 * (size_t)std::max(d.soft.nv, 0));
    tets.assign(d.soft.tets, d.soft.tets + 4 * (size_t)std::max(d.soft.nt, 0));
    if (d.soft.dirichlet) {
      has_dirichlet = true;
      dirichlet.assign(d.soft.dirichlet, d.soft.dirichlet + std::max(d.soft.nv, 0));
      for (uint8_t f : dirichlet) n_moving += f == 2;
    }
    for (int b = 0; b < d.n_bodies; ++b) {
      const taccel_body_desc& B = d.bodies[b];
      bverts.emplace_back(B.verts, B.verts + 3 * (size_t)B.nv);
      btris.emplace_back(B.tris, B.tris + 3 * (size_t)B.nf);
    }
    bodies.resize(d.n_bodies);
    for (int b = 0; b < d.n_bodies; ++b) {
      bodies[b] = d.bodies[b];
      bodies[b].verts = bverts[b].data();
      bodies[b].tris = btris[b].data();
    }
    desc.soft.verts = verts.data();
    desc.soft.tets = tets.data();
    desc.soft.dirichlet = has_dirichlet ? dirichlet.data() : nullptr;
    desc.bodies = bodies.empty() ? nullptr : bodies.data();
  }
};

struct Request {
  uint64_t id = 0;
  std::unique_ptr<OwnedScene> scene;
  int n_steps = 0, steps_done = 0;
  std::vector<double> body_targets;  // [n_steps][nb][12]
  std::vector<double> dir_targets;   // [n_steps][n_moving][3]
  size_t footprint = 0;
  int status = TACCEL_OK;
  bool finished = false;
  Clock::time_point t_submit, t_admit, t_done;
  std::vector<double> step_ms;
  std::map<int, std::vector<double>> fields;  // final state by taccel_field
};

// Conservative device footprint of a scene before it is built: node and tet data, the
// static pattern, per-tet Hessian blocks, contact primitives and their hash entries.
size_t estimate_footprint(const taccel_scene_desc& d) {
  size_t nodes = (size_t)d.soft.nv + 4 * (size_t)d.n_bodies + 4;
  size_t tets = (size_t)d.soft.nt;
  size_t prims = 0;
  for (int b = 0; b < d.n_bodies; ++b) prims += 3 * (size_t)d.bodies[b].nf + d.bodies[b].nv;
  prims += (size_t)d.soft.nv * 4;  // generous for the soft surface
  return 512 * nodes + 1800 * tets + 900 * prims + (4u << 20);
}

}  // namespace

struct Server {
  taccel_server_params params{};
  taccel_runtime rt{};
  bool has_rt = false;
  std::mutex mu;
  std::condition_variable cv_admit, cv_done;
  std::deque<Request*> pending;
  std::map<uint64_t, std::unique_ptr<Request>> requests;
  std::deque<uint64_t> completed;
  uint64_t next_id = 1;
  size_t used_bytes = 0;  // reservations of the running cohorts (never above the budget)
  size_t held_bytes = 0;  // what they hold now
  int running_cohorts = 0;
  bool stop = false;
  std::thread admit_thread;
  std::vector<std::thread> cohort_threads;
  std::atomic<size_t> peak_bytes{0};

  void finish(Request* r) {
    r->finished = true;
    r->t_done = Clock::now();
    completed.push_back(r->id);
    cv_done.notify_all();
  }

  // Host thread of one cohort.  Only this thread touches a running request's step data; the
  // request becomes visible to poll/read/release once finish() has run under the lock, after
  // which this thread no longer dereferences it (it may be released at any time).
  void run_cohort(std::vector<Request*> reqs, Batch* batch, size_t bytes) {
    size_t held = batch->device_bytes();
    bool refill_ok = reqs[0]->scene->desc.params.precision != TACCEL_MIXED;
    std::vector<int> done(reqs.size(), 0);
    for (;;) {
      const int n = (int)reqs.size();
      std::vector<int> mask(n, 1);
      std::vector<taccel_targets> tg(n);
      std::vector<taccel_status> per(n);
      std::vector<taccel_step_stats> st(n);
      {
        std::lock_guard<std::mutex> lk(mu);
        if (stop)
          for (int i = 0; i < n; ++i)
            if (!done[i]) {
              reqs[i]->status = TACCEL_CANCELLED;
              done[i] = 1;
              finish(reqs[i]);
            }
      }
      bool any = false;
      for (int i = 0; i < n; ++i) {
        mask[i] = !done[i];
        any = any || mask[i];
        if (!mask[i]) continue;
        Request* r = reqs[i];
        const int k = r->steps_done;
        const int nb = r->scene->desc.n_bodies, nm = r->scene->n_moving;
        tg[i].body_targets = nb ? r->body_targets.data() + (size_t)k * nb * 12 : nullptr;
        tg[i].dirichlet_targets = nm ? r->dir_targets.data() + (size_t)k * nm * 3 : nullptr;
      }
      if (!any) break;
      const auto t0 = Clock::now();
      batch->step(tg.data(), per.data(), st.data(), mask.data());
      const double dt = ms_since(t0, Clock::now());
      {
        // the cohort's buffers grow with its contacts, up to its reservation (the batch's
        // byte limit); the server's peak counts what the cohorts hold
        const size_t now = batch->device_bytes();
        std::lock_guard<std::mutex> lk(mu);
        held_bytes = held_bytes - held + now;
        held = now;
        peak_bytes = std::max(peak_bytes.load(), held_bytes);
      }
      bool freed = false;
      for (int i = 0; i < n; ++i) {
        if (!mask[i]) continue;
        Request* r = reqs[i];
        r->step_ms.push_back(dt);
        r->steps_done += 1;
        const bool failed = per[i] != TACCEL_OK;
        if (failed || r->steps_done >= r->n_steps) {
          if (failed) r->status = per[i];
          HostFields f = read_fields(batch, i, r);
          std::lock_guard<std::mutex> lk(mu);
          r->fields = std::move(f.fields);
          done[i] = 1;
          freed = true;
          finish(r);
        }
      }
      if (freed && refill_ok) refill(reqs, done, batch, bytes, held, refill_ok);
    }
    delete batch;
    std::lock_guard<std::mutex> lk(mu);
    used_bytes -= bytes;
    held_bytes -= held;
    running_cohorts -= 1;
    cv_admit.notify_all();
  }

  // Waiting requests take the slots that finished requests left in a running cohort: at a step
  // boundary the unfinished requests and newly admitted ones (arrival order, same precision,
  // within the cohort's reservation) form a new batch, into which the unfinished requests'
  // state moves bit for bit, so each continues exactly as it would have.  The old batch is
  // released before the new one is built, so the cohort never holds more than its reservation.
  // If the new batch cannot be built, the cohort goes on with its own requests and the new
  // ones go back to the front of the queue (the admission thread then forms cohorts for them).
  void refill(std::vector<Request*>& reqs, std::vector<int>& done, Batch*& batch, size_t bytes,
              size_t& held, bool& refill_ok) {
    std::vector<int> keep_idx;
    size_t need = 0;
    for (size_t i = 0; i < reqs.size(); ++i)
      if (!done[i]) {
        keep_idx.push_back((int)i);
        need += reqs[i]->footprint;
      }
    if (keep_idx.empty()) return;  // the cohort ends; admission forms new cohorts
    const int max_cohort = params.max_cohort > 0 ? params.max_cohort : 64;
    const int prec = reqs[keep_idx[0]]->scene->desc.params.precision;
    std::vector<Request*> add;
    {
      std::lock_guard<std::mutex> lk(mu);
      if (stop) return;
      while (!pending.empty() && (int)(keep_idx.size() + add.size()) < max_cohort) {
        Request* r = pending.front();
        if (r->scene->desc.params.precision != prec || need + r->footprint > bytes) break;
        pending.pop_front();
        need += r->footprint;
        add.push_back(r);
      }
    }
    if (add.empty()) return;
    std::vector<Batch::SceneState> states(keep_idx.size());
    std::vector<Request*> next;
    for (size_t j = 0; j < keep_idx.size(); ++j) {
      if (batch->export_state(keep_idx[j], states[j]) != TACCEL_OK) {
        // the state cannot be moved: the cohort goes on as it is
        std::lock_guard<std::mutex> lk(mu);
        for (auto it = add.rbegin(); it != add.rend(); ++it) pending.push_front(*it);
        refill_ok = false;
        cv_admit.notify_all();
        return;
      }
      next.push_back(reqs[keep_idx[j]]);
    }
    delete batch;
    batch = nullptr;
    taccel_runtime rt_local = rt;
    rt_local.stream = nullptr;
    auto build = [&](const std::vector<Request*>& rs) -> Batch* {
      std::vector<taccel_scene_desc> descs;
      for (Request* r : rs) descs.push_back(r->scene->desc);
      Batch* b = nullptr;
      std::string err;
      if (Batch::create(descs.data(), (int)descs.size(), has_rt ? &rt_local : nullptr, &b, err) != TACCEL_OK)
        return nullptr;
      return b;
    };
    std::vector<Request*> all = next;
    all.insert(all.end(), add.begin(), add.end());
    Batch* nb = build(all);
    if (!nb) {
      nb = build(next);  // the cohort's own requests, as before
      std::lock_guard<std::mutex> lk(mu);
      for (auto it = add.rbegin(); it != add.rend(); ++it) pending.push_front(*it);
      refill_ok = false;
      cv_admit.notify_all();
      all = next;
    } else {
      const auto now = Clock::now();
      for (Request* r : add) r->t_admit = now;
    }
    if (!nb) {  // the cohort's own scenes no longer build: they fail
      std::lock_guard<std::mutex> lk(mu);
      for (Request* r : next) {
        r->status = TACCEL_ERR_OOM;
        finish(r);
      }
      reqs.clear();
      done.clear();
      held_bytes -= held;
      held = 0;
      batch = nullptr;
      return;
    }
    nb->set_byte_limit(bytes);
    batch = nb;
    reqs = all;
    done.assign(reqs.size(), 0);
    for (size_t j = 0; j < next.size(); ++j)
      if (nb->import_state((int)j, states[j]) != TACCEL_OK) {  // cannot continue it exactly
        std::lock_guard<std::mutex> lk(mu);
        next[j]->status = TACCEL_ERR_HIP;
        done[j] = 1;
        finish(next[j]);
      }
    const size_t now_bytes = batch->device_bytes();
    std::lock_guard<std::mutex> lk(mu);
    held_bytes = held_bytes - held + now_bytes;
    held = now_bytes;
    peak_bytes = std::max(peak_bytes.load(), held_bytes);
  }

  struct HostFields {
    std::map<int, std::vector<double>> fields;
  };
  HostFields read_fields(Batch* batch, int i, Request* r) {
    HostFields out;
    const int nv = r->scene->desc.soft.nv, nb = r->scene->desc.n_bodies;
    const size_t counts[4] = {3 * (size_t)nv, 3 * (size_t)nv, 12 * (size_t)nb, 12 * (size_t)nb};
    for (int f = 0; f < 4; ++f) {
      std::vector<double> buf(counts[f]);
      if (batch->read(i, (taccel_field)f, buf.data(), buf.size() * sizeof(double)) == TACCEL_OK)
        out.fields[f] = std::move(buf);
    }
    return out;
  }

  void admission_loop() {
    const double budget = params.hbm_budget_bytes;
    const int max_cohort = params.max_cohort > 0 ? params.max_cohort : 64;
    const int max_cohorts = params.max_cohorts > 0 ? params.max_cohorts : 8;
    const auto coalesce = std::chrono::microseconds((long)(1000.0 * (params.coalesce_ms > 0 ? params.coalesce_ms : 1.0)));
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv_admit.wait(lk, [&] { return stop || (!pending.empty() && running_cohorts < max_cohorts); });
      if (stop) break;
      // let near-simultaneous arrivals join the same cohort
      lk.unlock();
      std::this_thread::sleep_for(coalesce);
      lk.lock();
      if (stop) break;
      std::vector<Request*> take;
      size_t bytes = 0;
      while (!pending.empty() && (int)take.size() < max_cohort) {
        Request* r = pending.front();
        // a batch computes in one precision; mixed precision runs one scene per batch
        if (!take.empty() && r->scene->desc.params.precision != take[0]->scene->desc.params.precision) break;
        if (!take.empty() && take[0]->scene->desc.params.precision == TACCEL_MIXED) break;
        if ((double)r->footprint > budget) {  // can never fit: fail it
          pending.pop_front();
          r->status = TACCEL_ERR_OOM;
          r->t_admit = Clock::now();
          finish(r);
          continue;
        }
        if ((double)(used_bytes + bytes + r->footprint) > budget) break;
        pending.pop_front();
        bytes += r->footprint;
        take.push_back(r);
      }
      if (take.empty()) {
        // wait for memory to free up
        cv_admit.wait(lk, [&] { return stop || running_cohorts == 0 || (!pending.empty() && (double)(used_bytes + pending.front()->footprint) <= budget); });
        continue;
      }
      used_bytes += bytes;
      running_cohorts += 1;
      lk.unlock();
      taccel_runtime rt_local = rt;
      rt_local.stream = nullptr;  // every cohort on a stream of its own
      auto create = [&](const std::vector<Request*>& rs, std::string& err) -> Batch* {
        std::vector<taccel_scene_desc> descs;
        for (Request* r : rs) descs.push_back(r->scene->desc);
        Batch* b = nullptr;
        const taccel_status st = Batch::create(descs.data(), (int)descs.size(), has_rt ? &rt_local : nullptr, &b, err);
        if (st != TACCEL_OK) {
          for (Request* r : rs) r->status = st;
          return nullptr;
        }
        return b;
      };
      std::string err;
      Batch* batch = create(take, err);
      std::vector<Request*> failed;
      if (!batch && take.size() > 1) {
        // one scene spoiled the cohort (e.g. it starts interpenetrating): find it alone
        std::vector<Request*> good;
        for (Request* r : take) {
          Batch* one = create({r}, err);
          if (one) {
            delete one;
            r->status = TACCEL_OK;
            good.push_back(r);
          } else {
            failed.push_back(r);
          }
        }
        take = good;
        batch = take.empty() ? nullptr : create(take, err);
        if (!batch) failed.insert(failed.end(), take.begin(), take.end());
      } else if (!batch) {
        failed = take;
      }
      const auto now = Clock::now();
      lk.lock();
      for (Request* r : take) r->t_admit = now;
      for (Request* r : failed) {
        r->t_admit = now;
        finish(r);
      }
      if (!batch) {
        used_bytes -= bytes;
        running_cohorts -= 1;
        continue;
      }
      // The cohort keeps its reservation: the batch may grow (contact pairs, candidates) up
      // to it and no further (a step that would needs more fails with ERR_OOM), so the
      // reservations of the running cohorts bound the device memory the server holds.  A
      // cohort whose creation already took more than its estimate is charged that instead.
      const size_t actual = batch->device_bytes();
      if (actual > bytes) {
        used_bytes += actual - bytes;
        bytes = actual;
      }
      batch->set_byte_limit(bytes);
      held_bytes += actual;
      peak_bytes = std::max(peak_bytes.load(), held_bytes);
      cohort_threads.emplace_back(&Server::run_cohort, this, take, batch, bytes);
    }
  }
};

}  // namespace tc

struct taccel_server {
  tc::Server s;
};

extern "C" {

taccel_status taccel_server_create(const taccel_server_params* p, const taccel_runtime* rt,
                                   taccel_server** out) {
  if (!p || !out || !(p->hbm_budget_bytes > 0)) {
    tc::set_last_error("server_create: params with hbm_budget_bytes > 0 and out required");
    return TACCEL_ERR_ARG;
  }
  taccel_server* srv = new taccel_server();
  srv->s.params = *p;
  if (rt) {
    srv->s.rt = *rt;
    srv->s.has_rt = true;
  }
  srv->s.admit_thread = std::thread(&tc::Server::admission_loop, &srv->s);
  *out = srv;
  return TACCEL_OK;
}

taccel_status taccel_server_submit(taccel_server* srv, const taccel_scene_desc* d, int32_t n_steps,
                                   const taccel_targets* per_step, uint64_t* req_id) {
  if (!srv || !d || n_steps <= 0 || !req_id) {
    tc::set_last_error("server_submit: bad arguments");
    return TACCEL_ERR_ARG;
  }
  {
    std::string err;
    const taccel_status st = tc::Batch::validate(d, 1, err);
    if (st != TACCEL_OK) {
      tc::set_last_error("server_submit: " + err);
      return st;
    }
  }
  auto r = std::make_unique<tc::Request>();
  r->scene = std::make_unique<tc::OwnedScene>(*d);
  r->n_steps = n_steps;
  const int nb = d->n_bodies, nm = r->scene->n_moving;
  bool any_prescribed = false;
  for (int b = 0; b < nb; ++b) any_prescribed = any_prescribed || d->bodies[b].prescribed;
  if ((any_prescribed || nm > 0) && !per_step) {
    tc::set_last_error("server_submit: per-step targets required");
    return TACCEL_ERR_ARG;
  }
  r->body_targets.assign((size_t)n_steps * nb * 12, 0.0);
  r->dir_targets.assign((size_t)n_steps * nm * 3, 0.0);
  for (int k = 0; per_step && k < n_steps; ++k) {
    if (nb && per_step[k].body_targets)
      std::memcpy(&r->body_targets[(size_t)k * nb * 12], per_step[k].body_targets, sizeof(double) * 12 * nb);
    if (nm) {
      if (!per_step[k].dirichlet_targets) {
        tc::set_last_error("server_submit: missing dirichlet_targets");
        return TACCEL_ERR_ARG;
      }
      std::memcpy(&r->dir_targets[(size_t)k * nm * 3], per_step[k].dirichlet_targets, sizeof(double) * 3 * nm);
    }
  }
  r->footprint = tc::estimate_footprint(*d);
  r->t_submit = tc::Clock::now();
  std::lock_guard<std::mutex> lk(srv->s.mu);
  r->id = srv->s.next_id++;
  *req_id = r->id;
  srv->s.pending.push_back(r.get());
  srv->s.requests.emplace(r->id, std::move(r));
  srv->s.cv_admit.notify_all();
  return TACCEL_OK;
}

taccel_status taccel_server_poll(taccel_server* srv, taccel_completion* out, int32_t cap, int32_t* n,
                                 int32_t wait_ms) {
  if (!srv || !n || (cap > 0 && !out)) {
    tc::set_last_error("server_poll: bad arguments");
    return TACCEL_ERR_ARG;
  }
  std::unique_lock<std::mutex> lk(srv->s.mu);
  if (srv->s.completed.empty() && wait_ms > 0)
    srv->s.cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !srv->s.completed.empty(); });
  int k = 0;
  while (k < cap && !srv->s.completed.empty()) {
    const uint64_t id = srv->s.completed.front();
    srv->s.completed.pop_front();
    const tc::Request& r = *srv->s.requests.at(id);
    taccel_completion& c = out[k++];
    c.req_id = id;
    c.status = r.status;
    c.n_steps = r.n_steps;
    c.steps_done = r.steps_done;
    c.wait_ms = tc::ms_since(r.t_submit, r.t_admit);
    c.run_ms = tc::ms_since(r.t_admit, r.t_done);
    double mean = 0.0, mx = 0.0;
    for (double v : r.step_ms) {
      mean += v;
      mx = std::max(mx, v);
    }
    c.mean_step_ms = r.step_ms.empty() ? 0.0 : mean / r.step_ms.size();
    c.max_step_ms = mx;
  }
  *n = k;
  return TACCEL_OK;
}

taccel_status taccel_server_step_latencies(taccel_server* srv, uint64_t req_id, double* out, int32_t cap,
                                           int32_t* n) {
  if (!srv || !n) return TACCEL_ERR_ARG;
  std::lock_guard<std::mutex> lk(srv->s.mu);
  auto it = srv->s.requests.find(req_id);
  if (it == srv->s.requests.end() || !it->second->finished) {
    tc::set_last_error("server_step_latencies: unknown or unfinished request");
    return TACCEL_ERR_ARG;
  }
  const auto& v = it->second->step_ms;
  *n = (int32_t)v.size();
  for (int k = 0; k < cap && k < (int)v.size(); ++k) out[k] = v[k];
  return TACCEL_OK;
}

taccel_status taccel_server_read(taccel_server* srv, uint64_t req_id, taccel_field f, void* dst, size_t bytes) {
  if (!srv) return TACCEL_ERR_ARG;
  std::lock_guard<std::mutex> lk(srv->s.mu);
  auto it = srv->s.requests.find(req_id);
  if (it == srv->s.requests.end() || !it->second->finished) {
    tc::set_last_error("server_read: unknown or unfinished request");
    return TACCEL_ERR_ARG;
  }
  auto fi = it->second->fields.find((int)f);
  if (fi == it->second->fields.end() || fi->second.size() * sizeof(double) != bytes || (bytes && !dst)) {
    tc::set_last_error("server_read: field not available or size mismatch");
    return TACCEL_ERR_ARG;
  }
  if (bytes) std::memcpy(dst, fi->second.data(), bytes);
  return TACCEL_OK;
}

taccel_status taccel_server_release(taccel_server* srv, uint64_t req_id) {
  if (!srv) return TACCEL_ERR_ARG;
  std::lock_guard<std::mutex> lk(srv->s.mu);
  auto it = srv->s.requests.find(req_id);
  if (it == srv->s.requests.end() || !it->second->finished) {
    tc::set_last_error("server_release: unknown or unfinished request");
    return TACCEL_ERR_ARG;
  }
  srv->s.requests.erase(it);
  return TACCEL_OK;
}

taccel_status taccel_server_info(taccel_server* srv, int32_t* queued, int32_t* running_cohorts,
                                 double* used_bytes, double* peak_bytes) {
  if (!srv) return TACCEL_ERR_ARG;
  std::lock_guard<std::mutex> lk(srv->s.mu);
  if (queued) *queued = (int32_t)srv->s.pending.size();
  if (running_cohorts) *running_cohorts = srv->s.running_cohorts;
  if (used_bytes) *used_bytes = (double)srv->s.used_bytes;
  if (peak_bytes) *peak_bytes = (double)srv->s.peak_bytes.load();
  return TACCEL_OK;
}

void taccel_server_destroy(taccel_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->s.mu);
    srv->s.stop = true;
    // queued requests that never started are completed as cancelled
    while (!srv->s.pending.empty()) {
      tc::Request* r = srv->s.pending.front();
      srv->s.pending.pop_front();
      r->status = TACCEL_CANCELLED;
      r->t_admit = tc::Clock::now();
      srv->s.finish(r);
    }
  }
  srv->s.cv_admit.notify_all();
  if (srv->s.admit_thread.joinable()) srv->s.admit_thread.join();
  for (auto& t : srv->s.cohort_threads)
    if (t.joinable()) t.join();
  delete srv;
}

}  // extern "C"
