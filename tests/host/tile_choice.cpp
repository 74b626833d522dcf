// Prints dmp::tile_choice for the queries read from stdin, one
// "kind S n forced_rb" per line (forced_rb 0: none): "rb split_tail" per line
// (host-only, no GPU).
#include <cstdio>

#include "plan.hpp"

int main() {
    int kind = 0, s = 0, n = 0, forced = 0;
    while (std::scanf("%d %d %d %d", &kind, &s, &n, &forced) == 4) {
        const dmp::TileChoice c = dmp::tile_choice(static_cast<dmp_kind>(kind), s, n, forced);
        std::printf("%d %d\n", c.rb, c.split_tail ? 1 : 0);
    }
    return 0;
}
