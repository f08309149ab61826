// Unit test of the server's admission and batching policy (CPU only).
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "serve_policy.hpp"

using namespace lscan::serve;

static int failures = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::printf("FAIL line %d: %s\n", __LINE__, #c);            \
            ++failures;                                                 \
        }                                                               \
    } while (0)

static PendingRequest req(uint64_t t, uint64_t key, uint64_t bytes) { return PendingRequest{t, key, bytes, t}; }
static std::vector<uint64_t> v(std::initializer_list<uint64_t> l) { return std::vector<uint64_t>(l); }

int main()
{
    {   // refusals
        Policy p(100, 2, 8);
        CHECK(p.submit(req(1, 1, 101)) == Admit::kTooLarge);
        CHECK(p.submit(req(2, 1, 100)) == Admit::kOk);
        CHECK(p.submit(req(3, 1, 1)) == Admit::kOk);
        CHECK(p.submit(req(4, 1, 1)) == Admit::kQueueFull);
        CHECK(p.pending() == 2);
    }
    {   // one batch per key, submit order kept
        Policy p(1000, 100, 100);
        p.submit(req(1, 7, 10));
        p.submit(req(2, 9, 10));
        p.submit(req(3, 7, 10));
        p.submit(req(4, 7, 10));
        Batch b = p.next_batch();
        CHECK(b.key == 7 && b.tickets == v({1, 3, 4}) && b.bytes == 30);
        b = p.next_batch();
        CHECK(b.key == 9 && b.tickets == v({2}));
        CHECK(p.next_batch().tickets.empty());
        CHECK(p.in_flight_bytes() == 40 && p.peak_bytes() == 40);
    }
    {   // budget: the oldest request waits for bytes, nothing of its key overtakes
        Policy p(100, 100, 100);
        p.submit(req(1, 1, 60));
        p.submit(req(2, 1, 50));
        p.submit(req(3, 1, 10));
        Batch b = p.next_batch();
        CHECK(b.tickets == v({1}));
        CHECK(p.next_batch().tickets.empty());  // 60 + 50 > 100: request 2 waits, 3 may not pass it
        p.release(60);
        b = p.next_batch();
        CHECK(b.tickets == v({2, 3}) && b.bytes == 60);
        CHECK(p.in_flight_bytes() == 60 && p.peak_bytes() == 60);
        p.release(60);
        CHECK(p.in_flight_bytes() == 0);
    }
    {   // another key may run while an older request of a different key waits? No: oldest first
        Policy p(100, 100, 100);
        p.submit(req(1, 1, 90));
        p.submit(req(2, 2, 50));
        p.submit(req(3, 2, 5));
        CHECK(p.next_batch().tickets == v({1}));
        CHECK(p.next_batch().tickets.empty());  // request 2 (oldest) needs 50 > 10 left
        p.release(90);
        Batch b = p.next_batch();
        CHECK(b.key == 2 && b.tickets == v({2, 3}));
    }
    {   // max_batch splits a long run of one key
        Policy p(1 << 30, 100, 2);
        for (uint64_t t = 1; t <= 5; ++t) p.submit(req(t, 3, 1));
        CHECK(p.next_batch().tickets == v({1, 2}));
        CHECK(p.next_batch().tickets == v({3, 4}));
        CHECK(p.next_batch().tickets == v({5}));
        CHECK(p.pending() == 0);
    }
    {   // release never underflows
        Policy p(10, 10, 10);
        p.release(5);
        CHECK(p.in_flight_bytes() == 0);
    }
    {   // large requests run alone, in submit order; smaller ones of the key are not grouped with them
        Policy p(1000, 100, 100, 100);
        p.submit(req(1, 1, 10));
        p.submit(req(2, 1, 150));   // solo
        p.submit(req(3, 1, 20));
        CHECK(!p.head_is_solo());
        Batch b = p.next_batch();
        CHECK(!b.solo && b.tickets == v({1, 3}));  // 2 is skipped: it never joins a batch
        CHECK(p.head_is_solo());
        b = p.next_batch();
        CHECK(b.solo && b.tickets == v({2}) && b.bytes == 150);
        CHECK(p.in_flight_bytes() == 180);
    }
    {   // a solo request still waits for budget like any other
        Policy p(200, 100, 100, 100);
        p.submit(req(1, 1, 90));
        p.submit(req(2, 2, 150));
        CHECK(p.next_batch().tickets == v({1}));
        CHECK(p.next_batch().tickets.empty());
        p.release(90);
        Batch b = p.next_batch();
        CHECK(b.solo && b.tickets == v({2}));
    }
    if (failures == 0) std::printf("serve policy: all checks passed\n");
    return failures == 0 ? 0 : 1;
}
