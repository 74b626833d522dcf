// Prints dmp::tile_choice for the queries read from stdin, one
// "kind S n" per line: "rb split_tail" per line (host-only, no GPU).
#include <cstdio>

#include "plan.hpp"

int main() {
    int kind = 0, s = 0, n = 0;
    while (std::scanf("%d %d %d", &kind, &s, &n) == 3) {
        const dmp::TileChoice c = dmp::tile_choice(static_cast<dmp_kind>(kind), s, n);
        std::printf("%d %d\n", c.rb, c.split_tail ? 1 : 0);
    }
    return 0;
}
