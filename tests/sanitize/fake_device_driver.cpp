// Host-side workout of the C ABI for sanitizer builds (AddressSanitizer +
// UndefinedBehaviorSanitizer, ThreadSanitizer). It needs no GPU: every server
// runs on the fake device (outputs in host memory, a timer or a host thread
// standing in for the kernels), and the plain and batch calls are driven only
// into their argument checks. Several threads submit, wait, poll, release and
// read statistics at once, so the scheduler's locking is exercised the way a
// serving process would.
//
// Exit status 0 when every scenario held; each failed check prints a line.
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include <unistd.h>

#include "tdct.h"

namespace tdct {
// Stores one autotune result under `key` and rewrites the cache file (the
// library's own entry point for its autotuner, declared here to drive the
// file code without a device).
void tune_cache_put(const std::string& key, const tdct_tune& t);
}

static std::atomic<int> g_failures{0};

#define CHECK(cond)                                                                        \
    do {                                                                                   \
        if (!(cond)) {                                                                     \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            g_failures++;                                                                  \
        }                                                                                  \
    } while (0)

static tdct_request make_req(int op, int w, int h) {
    tdct_request r;
    std::memset(&r, 0, sizeof r);
    r.op = op;
    r.w = w;
    r.h = h;
    r.keep = 64;
    r.input = reinterpret_cast<const void*>(uintptr_t(0x1000));  // never read by the fake device
    r.in_stride = w;
    for (int k = 0; k < 64; ++k) r.Q.q[k] = uint16_t(1 + (k % 9));
    return r;
}

static tdct_server_cfg make_cfg(int64_t budget, int fake_us) {
    tdct_server_cfg c;
    std::memset(&c, 0, sizeof c);
    c.budget_bytes = budget;
    c.streams = 4;
    c.max_batch = 8;
    c.batching = 1;
    c.fake_device_us = fake_us;
    return c;
}

static void sleep_us(int us) { std::this_thread::sleep_for(std::chrono::microseconds(us)); }

// Four threads submit and wait on their own requests, one releases nothing
// but reads statistics and polls foreign tickets all along.
static void stream_mode_many_threads(int streams, int max_wait_us) {
    tdct_server_cfg c = make_cfg(int64_t(1) << 24, 150);
    c.streams = streams;
    c.max_wait_us = max_wait_us;
    c.max_batch_px = 4 * 128 * 128;
    tdct_server* s = nullptr;
    CHECK(tdct_server_create(&c, &s) == TDCT_OK);
    if (!s) return;
    std::atomic<bool> stop{false};
    std::atomic<uint64_t> last_ticket{0};
    std::thread watcher([&] {
        while (!stop.load()) {
            tdct_stats st;
            CHECK(tdct_server_stats(s, &st) == TDCT_OK);
            CHECK(st.arena_high_water <= c.budget_bytes);
            tdct_result r;
            const int p = tdct_server_poll(s, last_ticket.load(), &r);
            CHECK(p == TDCT_OK || p == TDCT_EBUSY || p == TDCT_ENOTFOUND || p < 0);
            (void)tdct_server_last_error(s);
            sleep_us(50);
        }
    });
    std::vector<std::thread> clients;
    for (int t = 0; t < 4; ++t) {
        clients.emplace_back([&, t] {
            std::mt19937 rng(1234 + t);
            std::vector<uint64_t> mine;
            for (int k = 0; k < 120; ++k) {
                const int w = 8 * int(4 + rng() % 29), h = 8 * int(4 + rng() % 29);
                tdct_request r = make_req(int(rng() % 2), w, h);
                uint64_t tk = 0;
                CHECK(tdct_server_submit(s, &r, &tk) == TDCT_OK);
                last_ticket.store(tk);
                mine.push_back(tk);
                if (rng() % 4 == 0) sleep_us(int(rng() % 300));
                if (mine.size() >= 6) {  // wait for and release the oldest
                    tdct_result res;
                    CHECK(tdct_server_wait(s, mine.front(), &res) == TDCT_OK);
                    CHECK(res.status == TDCT_OK && res.output != nullptr);
                    CHECK(tdct_server_release(s, mine.front()) == TDCT_OK);
                    mine.erase(mine.begin());
                }
            }
            for (uint64_t tk : mine) {
                tdct_result res;
                CHECK(tdct_server_wait(s, tk, &res) == TDCT_OK && res.status == TDCT_OK);
                CHECK(tdct_server_release(s, tk) == TDCT_OK);
            }
        });
    }
    for (auto& th : clients) th.join();
    stop = true;
    watcher.join();
    tdct_stats st;
    CHECK(tdct_server_stats(s, &st) == TDCT_OK);
    CHECK(st.completed == 480 && st.failed == 0 && st.arena_bytes_in_use == 0);
    tdct_server_destroy(s);
}

// Injected failures at completion (n > 0) and partway through a launch
// (n < 0): failed requests give their memory back, the rest complete.
static void failures(int every) {
    tdct_server_cfg c = make_cfg(int64_t(1) << 22, 200);
    c.streams = 2;
    c.max_batch = 1;
    c.fake_fail_every = every;
    tdct_server* s = nullptr;
    CHECK(tdct_server_create(&c, &s) == TDCT_OK);
    if (!s) return;
    std::vector<uint64_t> tk(12);
    for (auto& t : tk) {
        tdct_request r = make_req(TDCT_OP_DECODE, 32, 32);
        CHECK(tdct_server_submit(s, &r, &t) == TDCT_OK);
    }
    CHECK(tdct_server_drain(s) == TDCT_OK);
    int ok = 0, bad = 0;
    for (uint64_t t : tk) {
        tdct_result r;
        CHECK(tdct_server_poll(s, t, &r) == TDCT_OK);
        (r.status == TDCT_OK ? ok : bad)++;
        CHECK(tdct_server_release(s, t) == TDCT_OK);
    }
    const int n = every > 0 ? every : -every;
    CHECK(bad == 12 / n && ok == 12 - 12 / n);
    tdct_stats st;
    CHECK(tdct_server_stats(s, &st) == TDCT_OK && st.arena_bytes_in_use == 0);
    tdct_server_destroy(s);
}

// A budget of three outputs: submitters block in admission while a
// releasing thread frees outputs as they complete.
static void budget_pressure() {
    const int64_t one = 64 * 64 * 2;
    tdct_server_cfg c = make_cfg(3 * one, 300);
    tdct_server* s = nullptr;
    CHECK(tdct_server_create(&c, &s) == TDCT_OK);
    if (!s) return;
    std::vector<uint64_t> tk(30);
    std::thread sub([&] {
        for (auto& t : tk) {
            tdct_request r = make_req(TDCT_OP_ENCODE, 64, 64);
            CHECK(tdct_server_submit(s, &r, &t) == TDCT_OK);
        }
    });
    sub.join();
    std::thread rel([&] {
        for (uint64_t t : tk) {
            tdct_result r;
            CHECK(tdct_server_wait(s, t, &r) == TDCT_OK && r.status == TDCT_OK);
            CHECK(tdct_server_release(s, t) == TDCT_OK);
        }
    });
    rel.join();
    tdct_stats st;
    CHECK(tdct_server_stats(s, &st) == TDCT_OK);
    CHECK(st.arena_high_water <= 3 * one && st.completed == 30);
    tdct_request big = make_req(TDCT_OP_ENCODE, 128, 128);
    uint64_t t = 0;
    CHECK(tdct_server_submit(s, &big, &t) == TDCT_ENOMEM);
    tdct_server_destroy(s);
}

// Open-loop replay, then shutdown with requests still in flight, then a
// shutdown with an output the client never released (the next request can
// never be admitted and is failed by destroy). No call overlaps destroy: the
// server is gone when it returns.
static void replay_and_shutdown() {
    tdct_server_cfg c = make_cfg(int64_t(1) << 24, 400);
    c.streams = 2;
    tdct_server* s = nullptr;
    CHECK(tdct_server_create(&c, &s) == TDCT_OK);
    if (!s) return;
    std::vector<tdct_request> reqs;
    std::vector<double> arr;
    for (int k = 0; k < 60; ++k) {
        reqs.push_back(make_req(k % 2, 32, 64));
        arr.push_back(150.0 * k);
    }
    std::vector<double> lat(60);
    std::vector<int32_t> st(60), bs(60);
    CHECK(tdct_server_replay(s, reqs.data(), arr.data(), 60, 0, nullptr, lat.data(), st.data(),
                             bs.data()) == TDCT_OK);
    for (int k = 0; k < 60; ++k) CHECK(st[k] == TDCT_OK && lat[k] >= 400 && bs[k] >= 1);
    for (int k = 0; k < 12; ++k) {
        uint64_t t;
        tdct_request r = make_req(TDCT_OP_ENCODE, 64, 64);
        CHECK(tdct_server_submit(s, &r, &t) == TDCT_OK);
    }
    tdct_server_destroy(s);  // drains the twelve in flight

    tdct_server_cfg c2 = make_cfg(64 * 64 * 2, 50);
    c2.streams = 1;
    CHECK(tdct_server_create(&c2, &s) == TDCT_OK);
    if (!s) return;
    uint64_t t1 = 0, t2 = 0;
    tdct_request r = make_req(TDCT_OP_ENCODE, 64, 64);
    CHECK(tdct_server_submit(s, &r, &t1) == TDCT_OK);
    tdct_result res;
    CHECK(tdct_server_wait(s, t1, &res) == TDCT_OK);
    CHECK(tdct_server_submit(s, &r, &t2) == TDCT_OK);
    sleep_us(5000);
    tdct_result r2;
    CHECK(tdct_server_poll(s, t2, &r2) == TDCT_OK && r2.status == TDCT_EBUSY);  // waits for memory
    tdct_server_destroy(s);  // fails the request instead of waiting forever
}

// Resident mode: a host thread plays the kernel's side of the queue
// protocol and checks that no queue slot or ring entry is reused early.
static void resident_mode() {
    tdct_server_cfg c = make_cfg(int64_t(1) << 26, 60);
    c.resident = 1;
    c.resident_jobs = 8;
    c.resident_tiles = 32;
    c.resident_idle_us = 2000;
    tdct_server* s = nullptr;
    CHECK(tdct_server_create(&c, &s) == TDCT_OK);
    if (!s) return;
    std::vector<std::thread> clients;
    for (int t = 0; t < 3; ++t) {
        clients.emplace_back([&, t] {
            std::mt19937 rng(77 + t);
            for (int k = 0; k < 60; ++k) {
                const int w = 8 * int(4 + rng() % 29), h = 8 * int(4 + rng() % 29);
                tdct_request r = make_req(int(rng() % 2), w, h);
                uint64_t tk = 0;
                CHECK(tdct_server_submit(s, &r, &tk) == TDCT_OK);
                if (k % 5 == 4) sleep_us(3000);  // past the idle limit now and then: relaunches
                tdct_result res;
                CHECK(tdct_server_wait(s, tk, &res) == TDCT_OK && res.status == TDCT_OK);
                CHECK(tdct_server_release(s, tk) == TDCT_OK);
            }
        });
    }
    for (auto& th : clients) th.join();
    CHECK(std::strcmp(tdct_server_last_error(s), "") == 0);
    for (int k = 0; k < 10; ++k) {  // left in flight for destroy
        uint64_t tk;
        tdct_request r = make_req(TDCT_OP_ENCODE, 64, 64);
        CHECK(tdct_server_submit(s, &r, &tk) == TDCT_OK);
    }
    tdct_server_destroy(s);
}

// Creation failures (an arena that cannot be allocated) free what they built.
static void failed_create() {
    for (int resident = 0; resident < 2; ++resident) {
        tdct_server_cfg c = make_cfg(int64_t(1) << 62, 10);
        c.resident = resident;
        tdct_server* s = nullptr;
        CHECK(tdct_server_create(&c, &s) == TDCT_ENOMEM && s == nullptr);
    }
}

// Plain and batch calls stop at their argument checks before any device work.
static void argument_checks() {
    tdct_qtable q;
    for (int k = 0; k < 64; ++k) q.q[k] = 1;
    const void* fake = reinterpret_cast<const void*>(uintptr_t(0x10000));
    CHECK(tdct_quantise((const uint8_t*)fake, 8, 7, 8, &q, 64, (int16_t*)fake, nullptr) == TDCT_EDIM);
    CHECK(tdct_forward(nullptr, 8, 8, 8, (int32_t*)fake, nullptr) == TDCT_EINVAL);
    CHECK(tdct_inverse((const int16_t*)((const char*)fake + 4), &q, 8, 8, (uint8_t*)fake, 8, nullptr) ==
          TDCT_EINVAL);
    tdct_image_desc d[2];
    std::memset(d, 0, sizeof d);
    for (int k = 0; k < 2; ++k) {
        d[k].op = TDCT_OP_ROUNDTRIP;
        d[k].w = d[k].h = 64;
        d[k].keep = 64;
        d[k].src = (const uint8_t*)fake + k * 64 * 64;
        d[k].src_stride = 64;
        d[k].dst = (uint8_t*)fake + k * 64 * 64 + 32;  // overlaps an input span
        d[k].dst_stride = 64;
    }
    tdct_plan* p = nullptr;
    CHECK(tdct_batch_plan(d, 2, &q, 1, nullptr, &p) == TDCT_EINVAL && p == nullptr);
    for (int st = 0; st > -8; --st) CHECK(std::strcmp(tdct_strerror(st), "unknown status") != 0);
}

// The autotune cache file: a key far longer than any the library makes
// survives a rewrite, and entries another process wrote to the file since it
// was opened are merged in.
static void tune_cache_file() {
    const std::string path = "/tmp/tdct_tune_cache_driver_" + std::to_string((long)getpid()) + ".json";
    const std::string longkey(3000, 'k');
    auto write = [&](const std::string& entries) {
        FILE* f = std::fopen(path.c_str(), "wb");
        CHECK(f != nullptr);
        if (!f) return;
        std::fprintf(f, "{\n \"format\": \"tdct-autotune-1\",\n \"entries\": {%s\n }\n}\n", entries.c_str());
        std::fclose(f);
    };
    write("\n  \"" + longkey + "\": [4, 1, 2, 1, 0]");
    CHECK(tdct_tune_cache_open(path.c_str()) == TDCT_OK);
    tdct::tune_cache_put("driver-a", tdct_tune{2, 4096, 1, 0, 1});
    write("\n  \"" + longkey + "\": [4, 1, 2, 1, 0],\n  \"driver-other\": [1, 16, 1, 1, 1]");
    tdct::tune_cache_put("driver-b", tdct_tune{8, 1, 1, 1, 1});
    tdct_tune_cache_stats st;
    CHECK(tdct_tune_cache_info(&st) == TDCT_OK && st.entries == 4 && st.write_errors == 0);
    CHECK(tdct_tune_cache_open(path.c_str()) == TDCT_OK);  // the rewritten file parses
    CHECK(tdct_tune_cache_info(&st) == TDCT_OK && st.on == 1 && st.entries == 4);
    CHECK(tdct_tune_cache_open(nullptr) == TDCT_OK);
    std::remove(path.c_str());
}

#define RUN(call)                                              \
    do {                                                       \
        std::fprintf(stderr, "scenario: %s\n", #call);         \
        call;                                                  \
    } while (0)

int main() {
    RUN(argument_checks());
    RUN(failed_create());
    RUN(stream_mode_many_threads(4, 0));
    RUN(stream_mode_many_threads(2, 500));
    RUN(failures(3));
    RUN(failures(-2));
    RUN(budget_pressure());
    RUN(replay_and_shutdown());
    RUN(resident_mode());
    RUN(tune_cache_file());
    const int f = g_failures.load();
    std::printf("fake-device driver: %s (%d failed checks)\n", f ? "FAILED" : "ok", f);
    return f ? 1 : 0;
}
