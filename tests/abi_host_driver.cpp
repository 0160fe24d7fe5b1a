// Host-side driver of the C ABI for a sanitizer build (AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code of the library; see
// test_host_sanitizers.py).  It calls only what runs without a device:
// argument validation of every entry point that checks before touching the
// device, and the binomial checkpoint schedule of Griewank & Walther (the
// host's most intricate code: an explicit task stack and a slot pool), over
// many chain lengths and snapshot budgets.  Each schedule is replayed here to
// check its structure, so that a run which is clean under the sanitizers is
// also a run of correct schedules.  Prints "ok" and exits 0 on success.

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "pa.h"

static int failures = 0;
#define EXPECT(cond)                                                         \
    do {                                                                     \
        if (!(cond)) {                                                       \
            std::printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond);    \
            ++failures;                                                      \
        }                                                                    \
    } while (0)

// Replays a schedule of L segments under `slots` snapshot slots: every
// segment is reversed exactly once, last to first; an advance starts from a
// slot holding its first boundary (or from the live state), and slot ids stay
// inside the budget with slot 0 never overwritten; the advance count is the
// optimum the library reports.
static void check_schedule(int L, int slots) {
    int64_t n = -1;
    EXPECT(pa_checkpoint_schedule(L, slots, nullptr, 0, &n) == PA_OK);
    if (n <= 0) return;
    std::vector<int32_t> a(5 * (size_t)n, -7);
    int64_t n2 = -1;
    EXPECT(pa_checkpoint_schedule(L, slots, a.data(), n, &n2) == PA_OK && n2 == n);
    const int S = slots < L ? slots : L;
    std::vector<int> held(S, -1);   // boundary each slot holds
    held[0] = 0;
    int live = 0;                   // boundary of the live state (-1: none)
    int next_rev = L - 1;
    int64_t advances = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t* o = &a[5 * (size_t)i];
        const int kind = o[0], x = o[1], y = o[2], src = o[3], dst = o[4];
        EXPECT(kind == 0 || kind == 1);
        EXPECT(src >= -1 && src < S && dst >= -1 && dst < S && dst != 0);
        const int from = src < 0 ? live : held[src];
        EXPECT(from == x);
        if (kind == 0) {
            EXPECT(x < y && y <= L);
            advances += y - x;
            live = y;
            if (dst >= 0) held[dst] = y;
        } else {
            EXPECT(y == x + 1 && x == next_rev);
            --next_rev;
            live = -1;
        }
    }
    EXPECT(next_rev == -1);
    // the schedule attains the fewest advances (forward sweep included)
    int64_t best = -1;
    EXPECT(pa_checkpoint_advances(L, slots, &best) == PA_OK);
    EXPECT(advances == best);
}

int main() {
    // schedules: every short chain under every budget, and a few long ones
    for (int L = 1; L <= 80; ++L)
        for (int s = 1; s <= 10; ++s) check_schedule(L, s);
    check_schedule(5000, 3);
    check_schedule(100000, 20);
    check_schedule(1 << 16, 1 << 16);

    int64_t n = 0, adv = 0;
    int32_t small[5];
    EXPECT(pa_checkpoint_schedule(0, 3, nullptr, 0, &n) == PA_EINVAL);
    EXPECT(pa_checkpoint_schedule(6, 0, nullptr, 0, &n) == PA_EINVAL);
    EXPECT(pa_checkpoint_schedule(6, 2, small, 1, &n) == PA_EINVAL && n > 1);
    EXPECT(pa_checkpoint_schedule(6, 2, nullptr, 0, nullptr) == PA_EINVAL);
    EXPECT(pa_checkpoint_schedule(PA_MAX_SCHEDULE_SEGMENTS + 1, 3, nullptr, 0, &n) == PA_EINVAL);
    EXPECT(std::strlen(pa_last_error()) > 0);
    EXPECT(pa_checkpoint_advances(0, 3, &adv) == PA_EINVAL);
    EXPECT(pa_checkpoint_advances(2000000000, 2, &adv) == PA_OK && adv > 0);
    EXPECT(pa_checkpoint_advances(2000000000, 2000000000, &adv) == PA_OK && adv == 2000000000 - 1);   // forward sweep only

    // validation that precedes every device call
    pa_physics good = {1e-3, 0.0, 5e-3, 0.0, 4, 0};
    pa_ctx* ctx = nullptr;
    const pa_physics bad_nu = {-1.0, 0.0, 5e-3, 0.0, 4, 0};
    const pa_physics bad_dt = {1e-3, 0.0, 0.0, 0.0, 4, 0};
    const pa_physics bad_kf = {1e-3, 0.0, 5e-3, 1.0, 40, 0};
    EXPECT(pa_create(&good, 7, 1, nullptr, &ctx) == PA_EINVAL && ctx == nullptr);
    EXPECT(pa_create(&good, 64, 0, nullptr, &ctx) == PA_EINVAL);
    EXPECT(pa_create(&good, 8, PA_MAX_MEMBERS + 1, nullptr, &ctx) == PA_EINVAL);
    EXPECT(pa_create(&bad_nu, 64, 1, nullptr, &ctx) == PA_EINVAL);
    EXPECT(pa_create(&bad_dt, 64, 1, nullptr, &ctx) == PA_EINVAL);
    EXPECT(pa_create(&bad_kf, 64, 1, nullptr, &ctx) == PA_EINVAL);
    EXPECT(pa_create(nullptr, 64, 1, nullptr, &ctx) == PA_EINVAL);
    EXPECT(pa_create(&good, 64, 1, nullptr, nullptr) == PA_EINVAL);
    EXPECT(pa_destroy(nullptr) == PA_OK);
    EXPECT(pa_set_stream(nullptr, nullptr) == PA_EINVAL);
    size_t bytes = 0;
    EXPECT(pa_workspace_bytes(nullptr, 10, 5, 0, 0, &bytes) == PA_EINVAL);
    pa_tiles t = {1, 2, 1, 2, 1, 2, 0};
    EXPECT(pa_set_tiles(nullptr, &t) == PA_EINVAL);
    EXPECT(pa_set_checkpoint_slots(nullptr, 2) == PA_EINVAL);
    EXPECT(pa_set_sobolev(nullptr, 1.0) == PA_EINVAL);
    EXPECT(pa_assimilate_state_bytes(nullptr, 3, 0, &bytes) == PA_EINVAL);
    EXPECT(pa_set_cancel_flags(nullptr, nullptr) == PA_EINVAL);
    double jh[4];
    int32_t it[1];
    pa_kernel k = {0, 0, 0.0};
    EXPECT(pa_assimilate_ex(nullptr, nullptr, 10, nullptr, &k, 0, 0, 3, 3, 5, jh, it, nullptr, nullptr, 0,
                            nullptr, 0) == PA_EINVAL);
    int32_t is_dev = -1;
    EXPECT(pa_is_device_memory(nullptr, &is_dev) == PA_OK && is_dev == 0);
    EXPECT(pa_is_device_memory(&good, nullptr) == PA_EINVAL);

    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
