// Launch schedule of the block PCG's inner loop on the concurrent paths (batch and
// server workers): chunks of four iterations captured once per solve as a hipGraph
// and replayed several times between host reads, the loop decisions taken on the
// device (LoopCtl). How many chunks run between two reads is chosen per size class
// by a small autotuner kept in the context.
#pragma once
#include <atomic>
#include <cmath>
#include <map>
#include <mutex>

namespace grass {

// chunks of four iterations replayed between two host reads; 0: kernel by kernel,
// the host reading the loop state every fourth iteration (as the plain path does)
constexpr int kSchedCand[] = {0, 1, 2, 4, 8};
constexpr int kSchedCands = 5;
constexpr int kSchedSamples = 3;  // inner phases timed per candidate before choosing

struct LaunchStats {
    std::atomic<long long> iterations{0}, host_reads{0}, replays{0}, captures{0};
};

struct Tuner {
    struct Cls {
        double sec[kSchedCands] = {};  // summed seconds per iteration
        int cnt[kSchedCands] = {};
        int choice = -1;
    };
    std::mutex mu;
    std::map<int, Cls> cls;

    // size class: node count in powers of two and the padded block width
    static int key(long long n, int kp) {
        return (int)std::lround(std::log2((double)(n > 1 ? n : 1))) * 256 + kp;
    }
    // candidate index for the next inner phase of this class
    int pick(int key_) {
        std::lock_guard<std::mutex> g(mu);
        Cls &c = cls[key_];
        if (c.choice >= 0) return c.choice;
        int best = 0;
        for (int i = 1; i < kSchedCands; i++)
            if (c.cnt[i] < c.cnt[best]) best = i;
        return best;
    }
    void record(int key_, int idx, double sec_per_iter) {
        std::lock_guard<std::mutex> g(mu);
        Cls &c = cls[key_];
        if (c.choice >= 0) return;
        c.sec[idx] += sec_per_iter;
        c.cnt[idx] += 1;
        for (int i = 0; i < kSchedCands; i++)
            if (c.cnt[i] < kSchedSamples) return;
        int best = 0;
        for (int i = 1; i < kSchedCands; i++)
            if (c.sec[i] / c.cnt[i] < c.sec[best] / c.cnt[best]) best = i;
        c.choice = best;
    }
};

struct LaunchSched {
    int mode = 0;    // 0: kernel by kernel; 1: captured chunks
    int chunks = 0;  // chunks between host reads; 0: chosen by the tuner
    Tuner *tuner = nullptr;
    LaunchStats *stats = nullptr;
};

// The schedule of the calling worker thread (null: kernel by kernel).
extern thread_local LaunchSched *g_sched;

}  // namespace grass
