// Host driver for the server's arena allocator (paper_1810_06800_amd/csrc/arena.h):
// reads "reset N", "alloc B", "free OFF B" and "stat" lines from stdin and
// prints one line per command, for tests/test_arena_cpu.py.
#include <cstdio>
#include <cstring>

#include "../paper_1810_06800_amd/csrc/arena.h"

int main()
{
    rsa::Arena a;
    char cmd[16];
    unsigned long long x, y;
    while (std::scanf("%15s", cmd) == 1) {
        if (!std::strcmp(cmd, "reset") && std::scanf("%llu", &x) == 1) {
            a.reset(x);
            std::printf("size %llu\n", (unsigned long long)a.size());
        } else if (!std::strcmp(cmd, "alloc") && std::scanf("%llu", &x) == 1) {
            uint64_t off = 0;
            if (a.alloc(x, off))
                std::printf("ok %llu\n", (unsigned long long)off);
            else
                std::printf("full\n");
        } else if (!std::strcmp(cmd, "free") && std::scanf("%llu %llu", &x, &y) == 2) {
            a.release(x, y);
            std::printf("freed\n");
        } else if (!std::strcmp(cmd, "stat")) {
            std::printf("stat %llu %llu %llu %llu\n", (unsigned long long)a.used(),
                        (unsigned long long)a.peak(), (unsigned long long)a.largest_free(),
                        (unsigned long long)a.free_ranges());
        } else {
            return 2;
        }
    }
    return 0;
}
