// barrier_model.cpp -- TEST INFRASTRUCTURE: a CPU model, with threads and
// C++ atomics, of the grid barrier protocol of the persistent ensemble launch
// (arrival count, generation word, status word; the last arrival resets the
// count and releases the next generation; a wait polls the generation with
// acquire loads and gives up after a bounded number of polls, or as soon as
// the status is set, and sets the status).  Each thread stands for one
// workgroup.  The memory orders are those of the device code (acq_rel
// arrival, release of the generation, acquire polls), so a missing fence in
// the protocol shows up here as a stale read under the C++ model.
//
//   barrier_model ok <threads> <rounds>
//       every thread writes its slot before each barrier and reads every
//       slot after it: all must hold the round number; exit 0 if so
//   barrier_model absent <threads> <poll_limit>
//       thread 0 never arrives at the first barrier: every other thread's
//       wait must give up (status set), later barriers must return at once,
//       and the program must end; prints the status and exits 0 if so
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <thread>
#include <vector>

struct Bar {
    std::atomic<unsigned> count{0}, gen{0}, status{0};
};

static bool grid_barrier(Bar &b, unsigned n, unsigned &gen, long long limit)
{
    const unsigned target = gen + 1;
    bool ok = true;
    const unsigned prev = b.count.fetch_add(1, std::memory_order_acq_rel);
    if (prev == n - 1) {
        b.count.store(0, std::memory_order_relaxed);
        b.gen.store(target, std::memory_order_release);
    } else {
        long long polls = 0;
        while (b.gen.load(std::memory_order_acquire) != target) {
            if (b.status.load(std::memory_order_relaxed) != 0 || ++polls > limit) {
                b.status.store(1, std::memory_order_relaxed);
                ok = false;
                break;
            }
            std::this_thread::yield();
        }
    }
    if (ok && b.status.load(std::memory_order_relaxed) != 0) ok = false;
    gen = target;
    return ok;
}

int main(int argc, char **argv)
{
    if (argc < 4) return 2;
    const std::string mode = argv[1];
    const unsigned n = (unsigned)atoi(argv[2]);
    Bar bar;
    if (mode == "ok") {
        const int rounds = atoi(argv[3]);
        std::vector<unsigned> slot(n, 0);            // plain (non-atomic) data, as the state is
        std::atomic<int> bad{0};
        std::vector<std::thread> th;
        for (unsigned t = 0; t < n; ++t)
            th.emplace_back([&, t] {
                unsigned gen = 0;
                for (int r = 1; r <= rounds; ++r) {
                    slot[t] = (unsigned)r;
                    if (!grid_barrier(bar, n, gen, 1ll << 40)) { bad++; return; }
                    for (unsigned k = 0; k < n; ++k)
                        if (slot[k] != (unsigned)r) bad++;
                    // a second barrier before the slots are written again
                    if (!grid_barrier(bar, n, gen, 1ll << 40)) { bad++; return; }
                }
            });
        for (auto &x : th) x.join();
        printf("ok rounds=%d threads=%u bad=%d status=%u\n", rounds, n, bad.load(), bar.status.load());
        return (bad.load() == 0 && bar.status.load() == 0) ? 0 : 1;
    }
    if (mode == "absent") {
        const long long limit = atoll(argv[3]);
        std::atomic<int> gave_up{0}, later_false{0};
        std::vector<std::thread> th;
        for (unsigned t = 1; t < n; ++t)             // thread 0 never arrives
            th.emplace_back([&] {
                unsigned gen = 0;
                if (!grid_barrier(bar, n, gen, limit)) gave_up++;
                if (!grid_barrier(bar, n, gen, limit)) later_false++;
            });
        for (auto &x : th) x.join();
        printf("absent threads=%u gave_up=%d later_false=%d status=%u\n", n, gave_up.load(), later_false.load(),
               bar.status.load());
        return (gave_up.load() == (int)n - 1 && later_false.load() == (int)n - 1 && bar.status.load() == 1) ? 0 : 1;
    }
    return 2;
}
