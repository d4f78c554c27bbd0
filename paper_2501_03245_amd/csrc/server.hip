// Request server: continuous batching of MSM and ECDSA-verification requests
// on one GPU.
//
// Requests are queued as they arrive.  `slots` worker threads, each with its
// own library context (and so its own stream and scratch), take the oldest
// waiting kind of work and admit as many queued requests of that kind as fit
// the batch limits and (MSMs) whose batched call's planned scratch fits the
// slot's share of the HBM budget, then run them as one batched call
// (ecc_msm_batch over all admitted MSMs of one curve, or ecc_verify_batch over
// all admitted verifications).  A request that arrives while batches are on
// the GPU joins the next batch of the next free slot, so batches of different
// slots overlap on the device.  Bases registered with ecc_server_add_bases
// stay resident in device memory; MSM requests name a range of them, which
// the batched call reads in place.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ecc_mi.h"

namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int limbs_of(ecc_curve c) { return c == ECC_BLS12_381_G1 ? 6 : 4; }

struct Request {
  uint64_t ticket = 0;
  bool is_msm = false;
  ecc_curve curve = ECC_BN254_G1;
  const uint64_t* bases_dev = nullptr;  // first base of the request (resident set)
  size_t n = 0;
  std::vector<uint64_t> scalars;  // MSM
  uint8_t hash[32];               // verify
  uint64_t pub[8], sig[8];
  double t_submit = 0;
};

struct Result {
  bool done = false;
  ecc_status status = ECC_OK;
  std::vector<uint64_t> xy;
  uint8_t flag = 0;
  double latency_ms = 0;
};

struct Bases {
  ecc_curve curve;
  size_t n;
  void* dev = nullptr;
};

}  // namespace

struct ecc_server {
  int device = 0;
  ecc_server_cfg cfg{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request> queue;
  std::unordered_map<uint64_t, Result> results;
  std::vector<Bases> bases;
  std::vector<std::thread> workers;
  std::vector<ecc_ctx*> ctxs;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::string err;
  // statistics
  std::vector<double> lat_msm, lat_verify;
  uint64_t batches = 0, msm_points = 0;
  uint64_t budget_cuts = 0, nomem_splits = 0, max_queue = 0;
  double t_first = -1, t_last = 0;
  // test-only executor (no device): admission plan and batch runner
  bool test_mode = false;
  ecc_server_exec exec{};
};

namespace {

// Device scratch the slot's context would hold for an MSM batch of the
// first k requests of `cand` (all of one curve), from the library's own plan
// of the call.
size_t msm_batch_bytes(ecc_server* s, ecc_ctx* ctx, const std::vector<Request>& cand, size_t k) {
  if (s->test_mode) {
    std::vector<uint64_t> sizes(k);
    for (size_t j = 0; j < k; j++) sizes[j] = cand[j].n;
    return s->exec.msm_batch_bytes(s->exec.user, sizes.data(), k);
  }
  std::vector<uint64_t> offs(k + 1, 0);
  for (size_t j = 0; j < k; j++) offs[j + 1] = offs[j] + cand[j].n;
  ecc_opts o{uint32_t(ECC_BASES_PER_MSM), 0, nullptr};
  size_t b = 0;
  if (ecc_msm_batch_scratch_bytes(ctx, cand[0].curve, offs.data(), k, &o, &b) != ECC_OK) return SIZE_MAX;
  return b;
}

// One batch of one kind, formed under the lock.  MSMs are admitted while
// their points fit max_batch_points and the scratch of the batched call (as
// the library plans it) fits the slot's share of the HBM budget; the first
// request is always taken (if it alone does not fit, its call reports
// ECC_ERR_NOMEM).
void take_batch(ecc_server* s, ecc_ctx* ctx, size_t hbm_share, std::vector<Request>& out) {
  out.clear();
  if (s->queue.empty()) return;
  const bool msm = s->queue.front().is_msm;
  const ecc_curve curve = s->queue.front().curve;
  size_t points = 0;
  for (auto it = s->queue.begin(); it != s->queue.end();) {
    bool same = it->is_msm == msm && (!msm || it->curve == curve);
    if (!same) {
      ++it;
      continue;
    }
    if (msm) {
      if (points + it->n > s->cfg.max_batch_points && !out.empty()) break;
      points += it->n;
    } else if (out.size() >= s->cfg.max_batch_verify) {
      break;
    }
    out.push_back(std::move(*it));
    it = s->queue.erase(it);
  }
  if (!msm || hbm_share == 0 || out.size() <= 1 || msm_batch_bytes(s, ctx, out, out.size()) <= hbm_share) return;
  // the longest prefix that fits (at least one request); the rest go back
  // to the front of the queue in their order
  size_t lo = 1, hi = out.size() - 1;
  while (lo < hi) {
    const size_t mid = (lo + hi + 1) / 2;
    if (msm_batch_bytes(s, ctx, out, mid) <= hbm_share) lo = mid;
    else hi = mid - 1;
  }
  for (size_t j = out.size(); j-- > lo;) s->queue.push_front(std::move(out[j]));
  out.resize(lo);
  s->budget_cuts++;
}

// requests [a, b) of the batch as one ecc_msm_batch call, bases read in place
// from the resident sets; a call that runs out of device memory is split in
// halves and each half retried
void run_msm_range(ecc_server* s, ecc_ctx* ctx, hipStream_t hs, std::vector<Request>& batch, size_t a, size_t b,
                   void** dev_in, size_t* dev_cap, std::vector<Result>& res) {
  const ecc_curve curve = batch[a].curve;
  const int L = limbs_of(curve);
  const size_t m = b - a;
  if (s->test_mode) {
    std::vector<uint64_t> sizes(m);
    std::vector<uint8_t> fl(m, 0);
    for (size_t j = 0; j < m; j++) sizes[j] = batch[a + j].n;
    const ecc_status st = s->exec.run_batch(s->exec.user, 1, sizes.data(), m, fl.data());
    if (st == ECC_ERR_NOMEM && m > 1) {
      {
        std::lock_guard<std::mutex> lk(s->mu);
        s->nomem_splits++;
      }
      const size_t mid = a + m / 2;
      run_msm_range(s, ctx, hs, batch, a, mid, dev_in, dev_cap, res);
      run_msm_range(s, ctx, hs, batch, mid, b, dev_in, dev_cap, res);
      return;
    }
    for (size_t j = 0; j < m; j++) {
      Result& r = res[a + j];
      r.status = st;
      if (st == ECC_OK) {
        r.xy.assign(size_t(2 * L), 0);
        r.flag = fl[j];
      }
    }
    return;
  }
  std::vector<uint64_t> offs(m + 1, 0);
  std::vector<const uint64_t*> ptrs(m);
  for (size_t j = 0; j < m; j++) {
    offs[j + 1] = offs[j] + batch[a + j].n;
    ptrs[j] = batch[a + j].bases_dev;
  }
  const size_t total = offs[m];
  // device input: scalars (4 u64 per point), outputs
  const size_t need = total * 4 * 8 + m * (2 * L * 8 + 1) + 256;
  ecc_status st = ECC_OK;
  if (*dev_cap < need) {
    if (*dev_in) (void)hipFree(*dev_in);
    *dev_in = nullptr;
    *dev_cap = 0;
    if (hipMalloc(dev_in, need) != hipSuccess) {
      *dev_in = nullptr;
      st = ECC_ERR_NOMEM;
    } else {
      *dev_cap = need;
    }
  }
  uint64_t* d_scal = static_cast<uint64_t*>(*dev_in);
  uint64_t* d_out = d_scal + total * 4;
  uint8_t* d_inf = reinterpret_cast<uint8_t*>(d_out + m * 2 * L);
  std::vector<uint64_t> h_scal(total * 4);
  if (st == ECC_OK) {
    for (size_t j = 0; j < m; j++) memcpy(h_scal.data() + offs[j] * 4, batch[a + j].scalars.data(), batch[a + j].n * 32);
    if (total && hipMemcpyAsync(d_scal, h_scal.data(), total * 32, hipMemcpyHostToDevice, hs) != hipSuccess)
      st = ECC_ERR_DEVICE;
  }
  if (st == ECC_OK) {
    // the batch call runs on the same stream, after the copy above
    ecc_opts o{uint32_t(ECC_BASES_PER_MSM) | (s->cfg.use_graph ? uint32_t(ECC_USE_GRAPH) : 0u), 0, hs};
    st = ecc_msm_batch(ctx, curve, reinterpret_cast<const uint64_t*>(ptrs.data()), d_scal, offs.data(), m, d_out,
                       d_inf, &o);
  }
  if (st == ECC_ERR_NOMEM && m > 1) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->nomem_splits++;
    }
    const size_t mid = a + m / 2;
    run_msm_range(s, ctx, hs, batch, a, mid, dev_in, dev_cap, res);
    run_msm_range(s, ctx, hs, batch, mid, b, dev_in, dev_cap, res);
    return;
  }
  std::vector<uint64_t> h_out(m * 2 * L);
  std::vector<uint8_t> h_inf(m);
  if (st == ECC_OK && (hipMemcpyAsync(h_out.data(), d_out, m * 2 * L * 8, hipMemcpyDeviceToHost, hs) != hipSuccess ||
                       hipMemcpyAsync(h_inf.data(), d_inf, m, hipMemcpyDeviceToHost, hs) != hipSuccess ||
                       hipStreamSynchronize(hs) != hipSuccess))
    st = ECC_ERR_DEVICE;
  for (size_t j = 0; j < m; j++) {
    Result& r = res[a + j];
    r.status = st;
    if (st == ECC_OK) {
      r.xy.assign(h_out.begin() + j * 2 * L, h_out.begin() + (j + 1) * 2 * L);
      r.flag = h_inf[j];
    }
  }
}

void run_msm_batch(ecc_server* s, ecc_ctx* ctx, hipStream_t hs, std::vector<Request>& batch, void** dev_in,
                   size_t* dev_cap, std::vector<Result>& res) {
  res.assign(batch.size(), Result{});
  run_msm_range(s, ctx, hs, batch, 0, batch.size(), dev_in, dev_cap, res);
}

void run_verify_batch(ecc_server* s, ecc_ctx* ctx, hipStream_t hs, std::vector<Request>& batch,
                      std::vector<Result>& res) {
  const size_t m = batch.size();
  if (s->test_mode) {
    std::vector<uint64_t> sizes(m, 1);
    std::vector<uint8_t> fl(m, 0);
    const ecc_status st = s->exec.run_batch(s->exec.user, 0, sizes.data(), m, fl.data());
    res.assign(m, Result{});
    for (size_t j = 0; j < m; j++) {
      res[j].status = st;
      res[j].flag = st == ECC_OK ? fl[j] : 0;
    }
    return;
  }
  std::vector<uint8_t> h(m * 32), v(m);
  std::vector<uint64_t> q(m * 8), sg(m * 8);
  for (size_t j = 0; j < m; j++) {
    memcpy(&h[j * 32], batch[j].hash, 32);
    memcpy(&q[j * 8], batch[j].pub, 64);
    memcpy(&sg[j * 8], batch[j].sig, 64);
  }
  ecc_opts o{uint32_t(ECC_HOST_PTRS), 0, hs};
  ecc_status st = ecc_verify_batch(ctx, ECC_SECP256R1, h.data(), q.data(), sg.data(), m, v.data(), &o);
  (void)s;
  res.assign(m, Result{});
  for (size_t j = 0; j < m; j++) {
    res[j].status = st;
    res[j].flag = st == ECC_OK ? v[j] : 0;
  }
}

void worker(ecc_server* s, int slot) {
  ecc_ctx* ctx = s->ctxs[slot];
  const size_t share = s->cfg.hbm_budget_bytes / size_t(std::max(1, s->cfg.slots));
  void* dev_in = nullptr;
  size_t dev_cap = 0;
  std::vector<Request> batch;
  std::vector<Result> res;
  hipStream_t hs = nullptr;
  if (!s->test_mode) {
    (void)hipSetDevice(s->device);
    if (hipStreamCreateWithFlags(&hs, hipStreamNonBlocking) != hipSuccess) hs = nullptr;
  }
  while (true) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
      if (s->stop && s->queue.empty()) break;
      take_batch(s, ctx, share, batch);
    }
    if (batch.empty()) continue;
    if (!hs && !s->test_mode) {
      res.assign(batch.size(), Result{});
      for (Result& r : res) r.status = ECC_ERR_DEVICE;
    } else if (batch[0].is_msm) {
      run_msm_batch(s, ctx, hs, batch, &dev_in, &dev_cap, res);
    } else {
      run_verify_batch(s, ctx, hs, batch, res);
    }
    const double t = now_ms();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->batches++;
      for (size_t j = 0; j < batch.size(); j++) {
        Result& r = s->results[batch[j].ticket];
        r = std::move(res[j]);
        r.done = true;
        r.latency_ms = t - batch[j].t_submit;
        (batch[j].is_msm ? s->lat_msm : s->lat_verify).push_back(r.latency_ms);
        if (batch[j].is_msm) s->msm_points += batch[j].n;
      }
      s->t_last = t;
    }
    s->cv_done.notify_all();
  }
  if (dev_in) (void)hipFree(dev_in);
  if (hs) (void)hipStreamDestroy(hs);
}

ecc_status enqueue(ecc_server* s, Request&& r, uint64_t* ticket) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return ECC_ERR_ARG;
    r.ticket = s->next_ticket++;
    r.t_submit = now_ms();
    if (s->t_first < 0) s->t_first = r.t_submit;
    *ticket = r.ticket;
    s->results[r.ticket] = Result{};
    s->queue.push_back(std::move(r));
    s->max_queue = std::max<uint64_t>(s->max_queue, s->queue.size());
  }
  s->cv_work.notify_one();
  return ECC_OK;
}

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  size_t k = size_t(q * double(v.size() - 1) + 0.5);
  return v[std::min(k, v.size() - 1)];
}

}  // namespace

extern "C" {

ecc_status ecc_server_create(int hip_device, const ecc_server_cfg* cfg, ecc_server** out) {
  if (!out || !cfg) return ECC_ERR_ARG;
  *out = nullptr;
  if (cfg->slots < 1 || cfg->slots > 16 || cfg->max_batch_points == 0 || cfg->max_batch_verify == 0)
    return ECC_ERR_ARG;
  auto s = std::make_unique<ecc_server>();
  s->device = hip_device;
  s->cfg = *cfg;
  const size_t share = cfg->hbm_budget_bytes / size_t(cfg->slots);
  for (int i = 0; i < cfg->slots; i++) {
    ecc_ctx* c = nullptr;
    ecc_status st = ecc_ctx_create(hip_device, share, &c);
    if (st != ECC_OK) {
      for (ecc_ctx* x : s->ctxs) ecc_ctx_destroy(x);
      return st;
    }
    s->ctxs.push_back(c);
  }
  for (int i = 0; i < cfg->slots; i++) s->workers.emplace_back(worker, s.get(), i);
  *out = s.release();
  return ECC_OK;
}

ecc_status ecc_server_create_with_exec(const ecc_server_cfg* cfg, const ecc_server_exec* exec, ecc_server** out) {
  if (!out || !cfg || !exec || !exec->msm_batch_bytes || !exec->run_batch) return ECC_ERR_ARG;
  *out = nullptr;
  if (cfg->slots < 1 || cfg->slots > 16 || cfg->max_batch_points == 0 || cfg->max_batch_verify == 0)
    return ECC_ERR_ARG;
  auto s = std::make_unique<ecc_server>();
  s->cfg = *cfg;
  s->test_mode = true;
  s->exec = *exec;
  s->ctxs.assign(size_t(cfg->slots), nullptr);
  for (int i = 0; i < cfg->slots; i++) s->workers.emplace_back(worker, s.get(), i);
  *out = s.release();
  return ECC_OK;
}

void ecc_server_destroy(ecc_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (std::thread& t : s->workers) t.join();
  if (s->test_mode) {
    delete s;
    return;
  }
  for (ecc_ctx* c : s->ctxs) ecc_ctx_destroy(c);
  (void)hipSetDevice(s->device);
  for (Bases& b : s->bases)
    if (b.dev) (void)hipFree(b.dev);
  delete s;
}

const char* ecc_server_last_error(const ecc_server* s) { return s ? s->err.c_str() : "null server"; }

ecc_status ecc_server_add_bases(ecc_server* s, ecc_curve curve, const uint64_t* bases, size_t n, uint32_t* id) {
  if (!s || !id || (n && !bases)) return ECC_ERR_ARG;
  if (curve != ECC_BN254_G1 && curve != ECC_BLS12_381_G1) return ECC_ERR_UNSUPPORTED;
  const size_t bytes = n * 2 * limbs_of(curve) * 8;
  Bases b{curve, n, nullptr};
  if (s->test_mode) {
    std::lock_guard<std::mutex> lk(s->mu);
    *id = uint32_t(s->bases.size());
    s->bases.push_back(b);
    return ECC_OK;
  }
  if (hipSetDevice(s->device) != hipSuccess) return ECC_ERR_DEVICE;
  if (hipMalloc(&b.dev, std::max<size_t>(bytes, 256)) != hipSuccess) return ECC_ERR_NOMEM;
  if (n && hipMemcpy(b.dev, bases, bytes, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(b.dev);
    return ECC_ERR_DEVICE;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  *id = uint32_t(s->bases.size());
  s->bases.push_back(b);
  return ECC_OK;
}

ecc_status ecc_server_submit_msm(ecc_server* s, uint32_t bases_id, size_t first, size_t n, const uint64_t* scalars,
                                 uint64_t* ticket) {
  if (!s || !ticket || (n && !scalars)) return ECC_ERR_ARG;
  Request r;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (bases_id >= s->bases.size()) return ECC_ERR_ARG;
    const Bases& B = s->bases[bases_id];
    if (first > B.n || n > B.n - first) return ECC_ERR_ARG;
    r.curve = B.curve;
    r.bases_dev = B.dev ? static_cast<const uint64_t*>(B.dev) + first * 2 * limbs_of(B.curve) : nullptr;
  }
  if (n > s->cfg.max_batch_points) return ECC_ERR_ARG;
  r.is_msm = true;
  r.n = n;
  r.scalars.assign(scalars, scalars + 4 * n);
  return enqueue(s, std::move(r), ticket);
}

ecc_status ecc_server_submit_verify(ecc_server* s, const uint8_t* hash, const uint64_t* pubkey, const uint64_t* sig,
                                    uint64_t* ticket) {
  if (!s || !ticket || !hash || !pubkey || !sig) return ECC_ERR_ARG;
  Request r;
  r.is_msm = false;
  r.curve = ECC_SECP256R1;
  memcpy(r.hash, hash, 32);
  memcpy(r.pub, pubkey, 64);
  memcpy(r.sig, sig, 64);
  return enqueue(s, std::move(r), ticket);
}

ecc_status ecc_server_submit_verify_many(ecc_server* s, const uint8_t* hashes, const uint64_t* pubkeys,
                                         const uint64_t* sigs, size_t m, uint64_t* tickets) {
  if (!s || (m && (!hashes || !pubkeys || !sigs || !tickets))) return ECC_ERR_ARG;
  if (m == 0) return ECC_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return ECC_ERR_ARG;
    const double t = now_ms();
    if (s->t_first < 0) s->t_first = t;
    for (size_t j = 0; j < m; j++) {
      Request r;
      r.is_msm = false;
      r.curve = ECC_SECP256R1;
      memcpy(r.hash, hashes + 32 * j, 32);
      memcpy(r.pub, pubkeys + 8 * j, 64);
      memcpy(r.sig, sigs + 8 * j, 64);
      r.ticket = s->next_ticket++;
      r.t_submit = t;
      tickets[j] = r.ticket;
      s->results[r.ticket] = Result{};
      s->queue.push_back(std::move(r));
    }
    s->max_queue = std::max<uint64_t>(s->max_queue, s->queue.size());
  }
  s->cv_work.notify_all();
  return ECC_OK;
}

ecc_status ecc_server_wait_many(ecc_server* s, const uint64_t* tickets, size_t m, uint8_t* flags,
                                double* latency_ms, int32_t* status) {
  if (!s || (m && !tickets)) return ECC_ERR_ARG;
  bool unknown = false;
  std::unique_lock<std::mutex> lk(s->mu);
  for (size_t j = 0; j < m; j++) {
    auto it = s->results.find(tickets[j]);
    if (it == s->results.end()) {
      unknown = true;
      if (status) status[j] = ECC_ERR_ARG;
      continue;
    }
    if (!it->second.done) {
      const uint64_t t = tickets[j];
      s->cv_done.wait(lk, [&] {
        auto f = s->results.find(t);
        return f == s->results.end() || f->second.done;
      });
      it = s->results.find(t);
      if (it == s->results.end()) {
        unknown = true;
        if (status) status[j] = ECC_ERR_ARG;
        continue;
      }
    }
    if (flags) flags[j] = it->second.flag;
    if (latency_ms) latency_ms[j] = it->second.latency_ms;
    if (status) status[j] = it->second.status;
    s->results.erase(it);
  }
  return unknown ? ECC_ERR_ARG : ECC_OK;
}

ecc_status ecc_server_wait(ecc_server* s, uint64_t ticket, int block, uint64_t* out_xy, uint8_t* out_flag,
                           double* latency_ms) {
  if (!s || !out_flag) return ECC_ERR_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->results.find(ticket);
  if (it == s->results.end()) return ECC_ERR_ARG;
  if (!it->second.done) {
    if (!block) return ECC_PENDING;
    // find(), not operator[]: a ticket taken meanwhile by another waiter
    // must not be re-inserted
    s->cv_done.wait(lk, [&] {
      auto f = s->results.find(ticket);
      return f == s->results.end() || f->second.done;
    });
    it = s->results.find(ticket);
    if (it == s->results.end()) return ECC_ERR_ARG;
  }
  Result r = std::move(it->second);
  s->results.erase(it);
  lk.unlock();
  if (r.status != ECC_OK) return r.status;
  if (out_xy && !r.xy.empty()) memcpy(out_xy, r.xy.data(), r.xy.size() * 8);
  *out_flag = r.flag;
  if (latency_ms) *latency_ms = r.latency_ms;
  return ECC_OK;
}

ecc_status ecc_server_get_stats(ecc_server* s, ecc_server_stats* out) {
  if (!s || !out) return ECC_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  ecc_server_stats st{};
  st.done_msm = s->lat_msm.size();
  st.done_verify = s->lat_verify.size();
  st.batches = s->batches;
  st.msm_points = s->msm_points;
  st.p50_msm_ms = percentile(s->lat_msm, 0.50);
  st.p99_msm_ms = percentile(s->lat_msm, 0.99);
  st.p50_verify_ms = percentile(s->lat_verify, 0.50);
  st.p99_verify_ms = percentile(s->lat_verify, 0.99);
  st.span_ms = s->t_first >= 0 ? s->t_last - s->t_first : 0.0;
  st.budget_cuts = s->budget_cuts;
  st.nomem_splits = s->nomem_splits;
  st.max_queue = s->max_queue;
  *out = st;
  return ECC_OK;
}

}  // extern "C"
