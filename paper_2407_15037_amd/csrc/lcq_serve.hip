// lcq_serve.hip -- continuous-batching request loop over the plain entry
// points: an open-loop schedule of quantize / dequantize requests is
// admitted as stream slots and device memory free up, runs concurrently on
// several HIP streams, and every output is compared on the device with the
// expected bytes the caller supplies.  Host side is a single native loop;
// nothing is allocated per request (outputs and workspaces are carved from a
// caller-owned device arena by a first-fit allocator).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <vector>

#include "lcq.h"
#include "lcq_host.hpp"
#include "lcq_tile.hpp"

using namespace lcq;

namespace {

// Count the 16-byte words of a[0..bytes) that differ from b (the tail is
// compared byte-wise); also flags a size mismatch against *size_dev.
__global__ __launch_bounds__(kBlock) void k_compare(const uint8_t *a, const uint8_t *b,
                                                    uint64_t bytes, const uint64_t *size_dev,
                                                    uint64_t want_size,
                                                    unsigned long long *mismatch) {
  unsigned long long bad = 0;
  const uint64_t nv = bytes / 16;
  const uint4 *va = reinterpret_cast<const uint4 *>(a);
  const uint4 *vb = reinterpret_cast<const uint4 *>(b);
  const uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint64_t gs = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = g; i < nv; i += gs) {
    const uint4 x = va[i], y = vb[i];
    bad += (x.x != y.x) | (x.y != y.y) | (x.z != y.z) | (x.w != y.w);
  }
  for (uint64_t i = nv * 16 + g; i < bytes; i += gs) bad += a[i] != b[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) bad += __shfl_xor(bad, o, 64);
  if ((threadIdx.x & 63) == 0 && bad) atomicAdd(mismatch, bad);
  if (g == 0 && size_dev && *size_dev != want_size) atomicAdd(mismatch, 1ull << 40);
}

__global__ void k_zero(unsigned long long *p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// First-fit allocator over [0, size) with 256-byte granules.
class Arena {
 public:
  explicit Arena(uint64_t size) { free_[0] = size; }
  bool alloc(uint64_t len, uint64_t *off) {
    len = (len + 255) & ~255ull;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= len) {
        *off = it->first;
        const uint64_t rest = it->second - len, start = it->first + len;
        free_.erase(it);
        if (rest) free_[start] = rest;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t len) {
    len = (len + 255) & ~255ull;
    auto it = free_.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<uint64_t, uint64_t> free_;  // offset -> length
};

uint64_t elem(lcq_dtype t) { return t == LCQ_F64 ? 8 : 4; }

// Device bytes a request needs: output, workspace and the size word.
uint64_t need_bytes(const lcq_request &r, uint64_t *out_len, uint64_t *ws_len) {
  if (r.op == 0) {
    *out_len = (lcq_max_stream_bytes(r.t, r.n) + 255) & ~255ull;
    *ws_len = (lcq_workspace_bytes(r.q, r.t, r.n) + 255) & ~255ull;
  } else {
    *out_len = (r.n * elem(r.t) + 255) & ~255ull;
    *ws_len = 256;
  }
  return *out_len + *ws_len + 256;
}

struct Running {
  uint32_t req;
  uint64_t off, len;
};

}  // namespace

extern "C" lcq_status lcq_serve(const lcq_server_config *cfg, const lcq_request *req, uint32_t nreq,
                                lcq_request_result *res) {
  if (!cfg || (nreq && (!req || !res))) return LCQ_ERR_ARG;
  if (cfg->n_streams == 0 || cfg->n_streams > 64 || !cfg->d_arena || !aligned16(cfg->d_arena))
    return LCQ_ERR_ARG;
  if (!cfg->d_scratch || cfg->scratch_bytes < 8ull * std::max<uint32_t>(nreq, 1)) return LCQ_ERR_CAPACITY;
  for (uint32_t i = 0; i < nreq; i++) {
    const lcq_request &R = req[i];
    if (R.op != 0 && R.op != 1) return LCQ_ERR_ARG;
    if (i && R.arrival_ns < req[i - 1].arrival_ns) return LCQ_ERR_ARG;
    if (R.t != LCQ_F32 && R.t != LCQ_F64) return LCQ_ERR_ARG;
    // the compare must stay inside the output buffer
    if (R.op == 0 && R.d_expect && R.expect_bytes > lcq_max_stream_bytes(R.t, R.n)) return LCQ_ERR_ARG;
  }
  // inputs, expected bytes and arena memory may still be produced (or, for
  // recycled memory, read) by work queued on other streams; the request
  // streams below do not order after them, so wait for it all first
  if (hipDeviceSynchronize() != hipSuccess) return LCQ_ERR_HIP;
  const uint32_t S = cfg->n_streams;
  std::vector<hipStream_t> streams(S, nullptr);
  std::vector<hipEvent_t> events(S, nullptr);
  lcq_status st = LCQ_OK;
  for (uint32_t s = 0; s < S && st == LCQ_OK; s++) {
    if (hipStreamCreateWithFlags(&streams[s], hipStreamNonBlocking) != hipSuccess) st = LCQ_ERR_HIP;
    else if (hipEventCreateWithFlags(&events[s], hipEventDisableTiming) != hipSuccess) st = LCQ_ERR_HIP;
  }
  auto cleanup = [&]() {
    for (uint32_t s = 0; s < S; s++) {
      if (events[s]) (void)hipEventDestroy(events[s]);
      if (streams[s]) (void)hipStreamDestroy(streams[s]);
    }
  };
  if (st != LCQ_OK) {
    cleanup();
    return st;
  }
  unsigned long long *mism = static_cast<unsigned long long *>(cfg->d_scratch);
  hipLaunchKernelGGL(k_zero, dim3(64), dim3(kBlock), 0, streams[0], mism, (uint64_t)nreq);
  if (hipStreamSynchronize(streams[0]) != hipSuccess) {
    cleanup();
    return LCQ_ERR_HIP;
  }
  for (uint32_t i = 0; i < nreq; i++) {
    res[i].admit_ns = res[i].done_ns = -1;
    res[i].mismatched = 0;
    res[i].status = LCQ_OK;
    res[i].stream = -1;
  }

  Arena arena(cfg->arena_bytes);
  uint8_t *base = static_cast<uint8_t *>(cfg->d_arena);
  std::deque<uint32_t> waiting;
  std::vector<int> busy(S, 0);
  std::vector<Running> run(S);
  uint32_t next = 0, finished = 0;
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  auto now_ns = [&]() {
    return (int64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(clk::now() - t0).count();
  };

  while (finished < nreq) {
    const int64_t t = now_ns();
    while (next < nreq && req[next].arrival_ns <= t) waiting.push_back(next++);
    // completions
    for (uint32_t s = 0; s < S; s++) {
      if (!busy[s]) continue;
      const hipError_t q = hipEventQuery(events[s]);
      if (q == hipErrorNotReady) continue;
      const uint32_t r = run[s].req;
      res[r].done_ns = now_ns();
      if (q != hipSuccess) res[r].status = LCQ_ERR_HIP;
      arena.release(run[s].off, run[s].len);
      busy[s] = 0;
      finished++;
    }
    // admissions, first come first served
    while (!waiting.empty()) {
      uint32_t s = 0;
      while (s < S && busy[s]) s++;
      if (s == S) break;
      const uint32_t r = waiting.front();
      const lcq_request &R = req[r];
      uint64_t out_len, ws_len, off;
      const uint64_t need = need_bytes(R, &out_len, &ws_len);
      if (need > cfg->arena_bytes) {  // can never fit
        waiting.pop_front();
        res[r].status = LCQ_ERR_CAPACITY;
        res[r].admit_ns = res[r].done_ns = now_ns();
        finished++;
        continue;
      }
      if (!arena.alloc(need, &off)) break;
      waiting.pop_front();
      uint8_t *out = base + off;
      uint8_t *ws = out + out_len;
      uint64_t *size_word = reinterpret_cast<uint64_t *>(ws + ws_len);
      res[r].admit_ns = now_ns();
      res[r].stream = (int32_t)s;
      lcq_status ls;
      if (R.op == 0) {
        ls = lcq_quantize(R.q, R.t, R.eb, R.d_in, R.n, out, out_len, size_word, ws, ws_len,
                          streams[s]);
      } else {
        ls = lcq_dequantize(R.t, R.d_in, R.in_bytes, out, R.n, ws, ws_len, streams[s]);
      }
      if (ls == LCQ_OK && R.d_expect) {
        const uint64_t bytes = R.op == 0 ? R.expect_bytes : R.n * elem(R.t);
        const uint64_t blocks = std::min<uint64_t>((bytes / 16 + kBlock - 1) / kBlock + 1, 1024);
        hipLaunchKernelGGL(k_compare, dim3((unsigned)blocks), dim3(kBlock), 0, streams[s], out,
                           static_cast<const uint8_t *>(R.d_expect), bytes,
                           R.op == 0 ? size_word : nullptr, R.expect_bytes, mism + r);
        if (hipGetLastError() != hipSuccess) ls = LCQ_ERR_HIP;
      }
      res[r].status = ls;
      if (hipEventRecord(events[s], streams[s]) != hipSuccess) res[r].status = LCQ_ERR_HIP;
      run[s] = Running{r, off, need};
      busy[s] = 1;
    }
  }
  for (uint32_t s = 0; s < S; s++) (void)hipStreamSynchronize(streams[s]);
  std::vector<unsigned long long> m(std::max<uint32_t>(nreq, 1), 0);
  if (nreq && hipMemcpy(m.data(), mism, 8ull * nreq, hipMemcpyDeviceToHost) != hipSuccess)
    st = LCQ_ERR_HIP;
  for (uint32_t i = 0; i < nreq; i++) res[i].mismatched = m[i];
  cleanup();
  return st;
}
