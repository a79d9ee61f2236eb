// Host-thread model of the persistent workers' synchronisation, for
// ThreadSanitizer and for randomised interleavings on the CPU (test
// infrastructure; it shares no code with the library, it restates the protocol):
//
//  * the two-level grid barrier: a workgroup reads its group's generation word,
//    counts itself in on its group counter (group = index mod 8); the last arrival
//    of a group resets that counter and counts the group in on the top counter; the
//    last group resets the top counter and writes generation + 1 to every group's
//    word; waiters spin until their group's word changes;
//  * a flat variant (cumulative group counters, zeroed before the launch; a waiter
//    spins until every group counter reaches its count for that barrier);
//  * the batch hand-off between the control workgroup and the compute workgroups:
//    the control side writes the batch descriptor (double-buffered by batch parity,
//    the next batch's written while the current one runs), broadcasts seq + 1 on
//    eight go words, and waits until every compute workgroup has counted the batch
//    done on its group's cumulative done counter.
//
// Workgroups are threads, device atomics are std::atomic (acquire/release where
// the device code fences). Every step may yield, at random, so runs differ in
// interleaving. Checks: nobody leaves barrier k before all arrived at it; every
// compute thread sees every batch's own descriptor, once, in order, unchanged
// while it works on it; no broadcast of batch k + 1 before every done of batch k.
// Any violation or a wait longer than the deadline exits non-zero with a message.
//
// usage: grid_protocol <threads> <rounds> <seed> <mode> [deadline_s]
//   mode: two-level | flat | handoff, or a planted mistake the checks must catch:
//   two-level-late-gen (the generation read after counting in) or
//   handoff-same-slot (the next batch's descriptor written into the current slot)
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

namespace {

struct alignas(64) Word {
  std::atomic<uint32_t> v{0};
};

std::atomic<bool> g_failed{false};
std::chrono::steady_clock::time_point g_deadline;

void fail(const char* what, long a, long b) {
  if (!g_failed.exchange(true)) std::fprintf(stderr, "FAILED: %s (%ld, %ld)\n", what, a, b);
}

// spin until pred() holds; false (and a failure) past the deadline
template <typename P>
bool spin_until(P pred, const char* what, long a) {
  while (!pred()) {
    if (g_failed.load(std::memory_order_relaxed)) return false;
    if (std::chrono::steady_clock::now() > g_deadline) {
      fail(what, a, -1);
      return false;
    }
    std::this_thread::yield();
  }
  return true;
}

struct Jitter {
  std::mt19937_64 rng;
  explicit Jitter(uint64_t s) : rng(s) {}
  void maybe_yield() {
    if ((rng() & 3) == 0) std::this_thread::yield();
  }
};

// ---------------------------------------------------------------- two-level barrier
struct TwoLevel {
  Word group[8], top, gen[8];
  uint32_t n;
  bool late_gen = false;          // planted mistake
  explicit TwoLevel(uint32_t n_) : n(n_) {}
  uint32_t members(uint32_t g) const { return (n - g + 7) >> 3; }
  uint32_t ngroups() const { return n < 8 ? n : 8; }
  // returns the generation to wait on, or UINT32_MAX when this thread released
  uint32_t arrive(uint32_t wg, Jitter& j) {
    const uint32_t g = wg & 7;
    uint32_t gen0 = late_gen ? 0 : gen[g].v.load(std::memory_order_relaxed);
    j.maybe_yield();
    const uint32_t prev = group[g].v.fetch_add(1, std::memory_order_acq_rel);
    if (late_gen) {
      j.maybe_yield();
      gen0 = gen[g].v.load(std::memory_order_relaxed);
    }
    if (prev != members(g) - 1) return gen0;
    j.maybe_yield();
    group[g].v.store(0, std::memory_order_relaxed);
    const uint32_t t = top.v.fetch_add(1, std::memory_order_acq_rel);
    if (t != ngroups() - 1) return gen0;
    j.maybe_yield();
    top.v.store(0, std::memory_order_relaxed);
    for (uint32_t q = 0; q < ngroups(); ++q) {
      gen[q].v.store(gen0 + 1, std::memory_order_release);
      j.maybe_yield();
    }
    return UINT32_MAX;
  }
  bool wait(uint32_t wg, uint32_t gen0, long round) {
    if (gen0 == UINT32_MAX) return true;
    const uint32_t g = wg & 7;
    return spin_until([&] { return gen[g].v.load(std::memory_order_acquire) != gen0; }, "two-level barrier wait",
                      round);
  }
};

// ---------------------------------------------------------------- flat barrier
struct Flat {
  Word group[8];
  uint32_t n;
  explicit Flat(uint32_t n_) : n(n_) {}
  uint32_t members(uint32_t g) const { return (n - g + 7) >> 3; }
  bool barrier(uint32_t wg, long round, Jitter& j) {
    group[wg & 7].v.fetch_add(1, std::memory_order_acq_rel);
    j.maybe_yield();
    return spin_until(
        [&] {
          for (uint32_t q = 0; q < 8 && q < n; ++q)
            if (group[q].v.load(std::memory_order_acquire) < (uint32_t)(round + 1) * members(q)) return false;
          return true;
        },
        "flat barrier wait", round);
  }
};

int run_barrier(uint32_t n, long rounds, uint64_t seed, bool flat, bool late_gen) {
  TwoLevel two(n);
  two.late_gen = late_gen;
  Flat fl(n);
  std::vector<std::atomic<uint32_t>> arrived(rounds);
  for (auto& a : arrived) a.store(0);
  std::vector<std::thread> ts;
  for (uint32_t wg = 0; wg < n; ++wg)
    ts.emplace_back([&, wg] {
      Jitter j(seed * 1000003 + wg);
      for (long k = 0; k < rounds && !g_failed.load(); ++k) {
        arrived[k].fetch_add(1, std::memory_order_acq_rel);
        bool ok;
        if (flat) {
          ok = fl.barrier(wg, k, j);
        } else {
          const uint32_t g0 = two.arrive(wg, j);
          j.maybe_yield();
          ok = two.wait(wg, g0, k);
        }
        if (!ok) return;
        const uint32_t a = arrived[k].load(std::memory_order_acquire);
        if (a != n) fail("left a barrier before everyone arrived", k, a);
      }
    });
  for (auto& t : ts) t.join();
  return g_failed.load() ? 1 : 0;
}

// ---------------------------------------------------------------- go / done hand-off
int run_handoff(uint32_t n, long batches, uint64_t seed, bool same_slot) {
  Word go[8], done[8];
  std::atomic<long> desc[2];
  desc[0].store(-1);
  desc[1].store(-1);
  std::atomic<long> started{-1};            // last batch broadcast
  std::vector<std::atomic<long>> seen(n);
  for (auto& s : seen) s.store(-1);
  auto members = [&](uint32_t g) { return (n - g + 7) >> 3; };
  std::vector<std::thread> ts;
  for (uint32_t wg = 0; wg < n; ++wg)
    ts.emplace_back([&, wg] {
      Jitter j(seed * 7919 + wg);
      const uint32_t g = wg & 7;
      for (long seq = 0; seq < batches && !g_failed.load(); ++seq) {
        if (!spin_until([&] { return go[g].v.load(std::memory_order_acquire) == (uint32_t)(seq + 1); }, "wait go",
                        seq))
          return;
        const long d = desc[seq & 1].load(std::memory_order_relaxed);
        if (d != seq) fail("compute thread read another batch's descriptor", seq, d);
        if (seen[wg].load() != seq - 1) fail("batch seen out of order", seq, seen[wg].load());
        seen[wg].store(seq);
        j.maybe_yield();
        if (desc[seq & 1].load(std::memory_order_relaxed) != seq) fail("descriptor changed during its batch", seq, 0);
        done[g].v.fetch_add(1, std::memory_order_acq_rel);
      }
    });
  std::thread ctl([&] {
    Jitter j(seed);
    desc[0].store(0, std::memory_order_relaxed);
    for (long seq = 0; seq < batches && !g_failed.load(); ++seq) {
      started.store(seq);
      for (uint32_t g = 0; g < 8; ++g) {
        go[g].v.store((uint32_t)(seq + 1), std::memory_order_release);
        j.maybe_yield();
      }
      // the next batch's descriptor now, while this one runs (its slot was last used
      // by batch seq - 1, which every compute thread has finished)
      if (seq + 1 < batches) desc[(seq + (same_slot ? 0 : 1)) & 1].store(seq + 1, std::memory_order_relaxed);
      for (uint32_t g = 0; g < 8 && g < n; ++g) {
        const uint32_t want = (uint32_t)(seq + 1) * members(g);
        if (!spin_until([&] { return done[g].v.load(std::memory_order_acquire) == want; }, "wait done", seq))
          return;
      }
      for (uint32_t wg = 0; wg < n; ++wg)
        if (seen[wg].load() != seq) fail("broadcast before a compute thread finished", seq, wg);
    }
  });
  ctl.join();
  for (auto& t : ts) t.join();
  return g_failed.load() ? 1 : 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 5 && argc != 6) {
    std::fprintf(stderr, "usage: %s <threads> <rounds> <seed> <mode> [deadline_s]\n", argv[0]);
    return 2;
  }
  const uint32_t n = (uint32_t)std::atoi(argv[1]);
  const long rounds = std::atol(argv[2]);
  const uint64_t seed = std::strtoull(argv[3], nullptr, 10);
  g_deadline = std::chrono::steady_clock::now() + std::chrono::seconds(argc == 6 ? std::atoi(argv[5]) : 60);
  const char* m = argv[4];
  int rc;
  if (!std::strcmp(m, "two-level")) rc = run_barrier(n, rounds, seed, false, false);
  else if (!std::strcmp(m, "two-level-late-gen")) rc = run_barrier(n, rounds, seed, false, true);
  else if (!std::strcmp(m, "flat")) rc = run_barrier(n, rounds, seed, true, false);
  else if (!std::strcmp(m, "handoff")) rc = run_handoff(n, rounds, seed, false);
  else if (!std::strcmp(m, "handoff-same-slot")) rc = run_handoff(n, rounds, seed, true);
  else return 2;
  if (!rc) std::printf("ok: %s, %u threads, %ld rounds\n", argv[4], n, rounds);
  return rc;
}
