// Host model of the trade kernel's help-job protocol (the tickets shared
// write phases and giant passes use): a ticket of generation (16 bits),
// chunk count (24) and next chunk (24); a claim loads the ticket, gives up
// when no chunk is left, else takes one with a fetch-and-add whose returned
// value alone says whether it holds a chunk; the owner opens a job (done and
// own counters reset, fields stored, then the ticket of a new generation,
// then its mask bit), claims chunks itself, clears the mask bit and waits
// until every chunk is reported done. Helpers look at the mask, claim, read
// the fields of the generation they hold a chunk of, work, and report done.
// A helper may take a run of chunks of one job in a row: it keeps the fields
// it read while the tickets it claims show the same generation, and reads
// them again when a claim shows a new one.
//
// Every thread yields at random points. The model checks that each chunk of
// each generation is worked exactly once, with that generation's fields, that
// no chunk beyond the count is ever worked, and that every wait ends (the
// program exits with a status; the test runs it under a time limit).
// It checks the protocol's interleavings, not the GPU's memory ordering.
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

constexpr int kCountBits = 24;
constexpr uint64_t kMask = (1ull << kCountBits) - 1;
constexpr int kMaxChunks = 12;

struct Job {
  std::atomic<uint64_t> ticket{0};
  std::atomic<int32_t> done{0};
  std::atomic<int32_t> fields_gen{0};   // the generation's fields (one word stands for all)
  std::atomic<int32_t> fields_chunks{0};
};

static uint32_t ticket_gen(uint64_t t) { return (uint32_t)(t >> (2 * kCountBits)); }
static int32_t ticket_chunks(uint64_t t) { return (int32_t)((t >> kCountBits) & kMask); }
static int32_t ticket_next(uint64_t t) { return (int32_t)(t & kMask); }

static thread_local std::mt19937_64 rng{std::random_device{}()};
static void jitter() {
  const uint64_t r = rng() & 63;
  if (r < 8) std::this_thread::yield();
  else if (r == 9) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 50));
}

static int32_t claim_chunk(Job& J, uint32_t* gen = nullptr) {
  const uint64_t seen = J.ticket.load(std::memory_order_relaxed);
  if (ticket_next(seen) >= ticket_chunks(seen)) return -1;
  jitter();
  const uint64_t t = J.ticket.fetch_add(1, std::memory_order_relaxed);
  if (gen) *gen = ticket_gen(t);
  return ticket_next(t) < ticket_chunks(t) ? ticket_next(t) : -1;
}

int main(int argc, char** argv) {
  const int owners = argc > 1 ? atoi(argv[1]) : 3;
  const int helpers = argc > 2 ? atoi(argv[2]) : 12;
  const int gens = argc > 3 ? atoi(argv[3]) : 20000;
  const int runs = argc > 4 ? atoi(argv[4]) : 1;   // chunks a helper takes in a row
  std::vector<Job> jobs(owners);
  std::atomic<uint32_t> mask{0};
  // worked[o][gen % 4096][chunk]: how often that chunk was worked
  std::vector<std::atomic<int32_t>> worked((size_t)owners * 4096 * kMaxChunks);
  for (auto& w : worked) w.store(0);
  std::atomic<int> bad{0}, stop{0};
  auto work = [&](int o, int32_t gen, int32_t chunks, int32_t c) {
    if (c >= chunks || gen <= 0) bad.fetch_add(1);
    else worked[((size_t)o * 4096 + (gen % 4096)) * kMaxChunks + c].fetch_add(1);
  };
  std::vector<std::thread> th;
  for (int o = 0; o < owners; ++o)
    th.emplace_back([&, o] {
      Job& J = jobs[o];
      for (int32_t gen = 1; gen <= gens; ++gen) {
        const int32_t chunks = 1 + (int32_t)(rng() % kMaxChunks);
        for (int c = 0; c < kMaxChunks; ++c)
          worked[((size_t)o * 4096 + (gen % 4096)) * kMaxChunks + c].store(0);
        // open: counters, fields, fence, ticket of the new generation, fence, mask bit
        J.done.store(0, std::memory_order_relaxed);
        J.fields_gen.store(gen, std::memory_order_relaxed);
        J.fields_chunks.store(chunks, std::memory_order_relaxed);
        std::atomic_thread_fence(std::memory_order_seq_cst);
        jitter();
        const uint64_t g = (ticket_gen(J.ticket.load(std::memory_order_relaxed)) + 1u) & 0xFFFFull;
        J.ticket.store((g << (2 * kCountBits)) | ((uint64_t)chunks << kCountBits), std::memory_order_relaxed);
        std::atomic_thread_fence(std::memory_order_seq_cst);
        mask.fetch_or(1u << o, std::memory_order_relaxed);
        // the owner's own claims
        for (;;) {
          const int32_t c = claim_chunk(J);
          if (c < 0) break;
          jitter();
          work(o, J.fields_gen.load(std::memory_order_relaxed), J.fields_chunks.load(std::memory_order_relaxed), c);
          std::atomic_thread_fence(std::memory_order_seq_cst);
          J.done.fetch_add(1, std::memory_order_relaxed);
        }
        // close: mask bit off, wait for every chunk
        mask.fetch_and(~(1u << o), std::memory_order_relaxed);
        const auto t0 = std::chrono::steady_clock::now();
        while (J.done.load(std::memory_order_relaxed) < chunks) {
          std::this_thread::yield();
          if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(20)) {
            fprintf(stderr, "owner %d generation %d: close never finished (done %d of %d)\n", o, gen,
                    J.done.load(), chunks);
            bad.fetch_add(1);
            stop.store(1);
            return;
          }
        }
        for (int c = 0; c < kMaxChunks; ++c) {
          const int32_t v = worked[((size_t)o * 4096 + (gen % 4096)) * kMaxChunks + c].load();
          if (v != (c < chunks ? 1 : 0)) {
            fprintf(stderr, "owner %d generation %d chunk %d worked %d times\n", o, gen, c, v);
            bad.fetch_add(1);
          }
        }
      }
    });
  for (int h = 0; h < helpers; ++h)
    th.emplace_back([&, h] {
      while (!stop.load(std::memory_order_relaxed)) {
        const uint32_t m = mask.load(std::memory_order_relaxed);
        if (!m) { std::this_thread::yield(); continue; }
        int pick = __builtin_ctz(m);
        for (int i = 0; i < owners; ++i)
          if ((m >> ((h + i) % owners)) & 1u) { pick = (h + i) % owners; break; }
        Job& J = jobs[pick];
        uint32_t gen = 0;
        int32_t c = claim_chunk(J, &gen);
        if (c < 0) continue;
        uint32_t have = 0;   // generation (with bit 16 set) whose fields are held
        int32_t fgen = 0, fchunks = 0;
        for (int run = 0;;) {
          std::atomic_thread_fence(std::memory_order_seq_cst);
          jitter();
          if (have != (gen | 0x10000u)) {
            fgen = J.fields_gen.load(std::memory_order_relaxed);
            fchunks = J.fields_chunks.load(std::memory_order_relaxed);
            have = gen | 0x10000u;
          }
          work(pick, fgen, fchunks, c);
          std::atomic_thread_fence(std::memory_order_seq_cst);
          jitter();
          J.done.fetch_add(1, std::memory_order_relaxed);
          if (++run >= runs) break;
          c = claim_chunk(J, &gen);
          if (c < 0) break;
        }
      }
    });
  for (int o = 0; o < owners; ++o) th[o].join();
  stop.store(1);
  for (size_t i = owners; i < th.size(); ++i) th[i].join();
  printf("%s: %d owners x %d generations, %d helpers, runs of %d\n", bad.load() ? "FAIL" : "ok", owners, gens,
         helpers, runs);
  return bad.load() ? 1 : 0;
}
