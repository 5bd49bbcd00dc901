// Host-side stress of the ring pipeline's bookkeeping in dry-run mode (no
// device work): producer threads acquire/publish bursts on their streams
// while a reader thread pops results, another thread polls the counters and
// the dispatcher completes bursts.  Built with the host sanitizers by the
// test that runs it; exits non-zero on any ordering or accounting error.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <thread>
#include <vector>

#include "combgpu.h"

namespace {

int fails = 0;

#define CHECK(cond, ...)                \
  do {                                  \
    if (!(cond)) {                      \
      std::fprintf(stderr, __VA_ARGS__); \
      std::fprintf(stderr, "\n");       \
      ++fails;                          \
    }                                   \
  } while (0)

void run(bool keep, int n_streams, int slots, int bursts_per_stream, double us_per_frame) {
  cg_pipeline* pipe = nullptr;
  cg_status st = cg_pipeline_create(n_streams, nullptr, nullptr, slots, 64,
                                    CG_PIPE_DRY_RUN | (keep ? CG_PIPE_KEEP_RESULTS : 0u),
                                    us_per_frame, &pipe);
  CHECK(st == CG_OK && pipe, "create failed: %d", st);
  if (!pipe) return;
  std::atomic<int> producers_left(n_streams);
  std::atomic<long> published(0), overflows(0), read_count(0);
  std::vector<std::thread> th;
  for (int s = 0; s < n_streams; ++s) {
    th.emplace_back([&, s] {
      for (int b = 0; b < bursts_per_stream; ++b) {
        int32_t slot = -1;
        void* buf = nullptr;
        for (;;) {
          const cg_status a = cg_pipeline_acquire(pipe, s, &slot, &buf);
          if (a == CG_OK) break;
          CHECK(a == CG_ERR_RING_FULL, "acquire: %d", a);
          overflows.fetch_add(1);
          std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
        const cg_status p = cg_pipeline_publish(pipe, s, slot, 1 + (b * 7 + s) % 64, b);
        CHECK(p == CG_OK, "publish: %d", p);
        published.fetch_add(1);
      }
      producers_left.fetch_sub(1);
    });
  }
  std::atomic<bool> stop_poll(false);
  std::thread poller([&] {
    double out[CG_PIPE_NSTATS];
    while (!stop_poll.load()) {
      CHECK(cg_pipeline_stats(pipe, out, CG_PIPE_NSTATS) == CG_OK, "stats");
      CHECK(out[5] <= out[6] + 1e-9 && out[6] <= out[7] + 1e-9, "latency order");
      std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
  });
  std::thread reader;
  if (keep) {
    reader = std::thread([&] {
      std::vector<int64_t> last(n_streams, -1);
      std::vector<float> params(64 * 4);
      std::vector<int32_t> status(64);
      long want = (long)n_streams * bursts_per_stream;
      const auto deadline = std::chrono::steady_clock::now() + std::chrono::seconds(120);
      while (read_count.load() < want) {
        if (std::chrono::steady_clock::now() > deadline) {
          CHECK(false, "reader: %ld of %ld bursts read before the deadline", read_count.load(),
                want);
          break;
        }
        bool any = false;
        for (int s = 0; s < n_streams; ++s) {
          int32_t n = 0;
          int64_t seq = -1;
          const cg_status r =
              cg_pipeline_read(pipe, s, params.data(), status.data(), 64, &n, &seq);
          if (r == CG_OK) {
            CHECK(seq == last[s] + 1, "stream %d: seq %lld after %lld", s, (long long)seq,
                  (long long)last[s]);
            CHECK(n == 1 + (int)((seq * 7 + s) % 64), "stream %d: n %d", s, n);
            last[s] = seq;
            read_count.fetch_add(1);
            any = true;
          } else {
            CHECK(r == CG_ERR_STATE && n == 0, "read: %d", r);
          }
        }
        if (!any) std::this_thread::sleep_for(std::chrono::microseconds(50));
      }
    });
  }
  for (auto& t : th) t.join();
  if (keep) reader.join();
  CHECK(cg_pipeline_drain(pipe, 20000) == CG_OK, "drain");
  stop_poll.store(true);
  poller.join();
  double out[CG_PIPE_NSTATS];
  CHECK(cg_pipeline_stats(pipe, out, CG_PIPE_NSTATS) == CG_OK, "stats");
  const long total = (long)n_streams * bursts_per_stream;
  CHECK((long)out[0] == total, "bursts %g != %ld", out[0], total);
  CHECK((long)out[3] == overflows.load(), "overflows %g != %ld", out[3], overflows.load());
  CHECK(published.load() == total, "published");
  CHECK(cg_pipeline_destroy(pipe) == CG_OK, "destroy");
  std::printf("keep=%d streams=%d slots=%d bursts=%ld overflows=%ld\n", keep ? 1 : 0, n_streams,
              slots, total, overflows.load());
}

}  // namespace

int main() {
  run(false, 4, 3, 400, 2.0);
  run(true, 6, 2, 300, 1.0);
  run(true, 3, 8, 500, 0.0);
  if (fails) {
    std::fprintf(stderr, "%d check(s) failed\n", fails);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
