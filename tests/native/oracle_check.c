/* Drives every entry point of the CPU oracle on small lattices, for builds
 * with AddressSanitizer and UndefinedBehaviorSanitizer (test code only).
 * Prints one line per case: "case <id> <digest> <mass> <px> <py> <swaps>
 * <block sum> <row sum>" and "OK" at the end; a sanitizer report or a bad
 * return code fails the run. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/fhp_oracle.h"

static int fails = 0;

static void expect(int ok, const char *what, int id) {
    if (!ok) {
        printf("case %d: %s\n", id, what);
        fails++;
    }
}

int main(void) {
    static const uint32_t sizes[][2] = {{2, 2}, {6, 4}, {64, 2}, {130, 6}, {192, 10}};
    static const uint32_t blocks[] = {1, 3, 16, 64, 200};
    int id = 0;
    for (int rules = 0; rules < 3; rules++) {
        uint8_t tab[128];
        expect(fhpo_rule_table(rules, 0, tab) == 0 && fhpo_rule_table(rules, 1, tab) == 0,
               "rule table", id);
        for (int chir = 0; chir < 3; chir++) {
            for (size_t k = 0; k < sizeof sizes / sizeof sizes[0]; k++, id++) {
                const uint32_t W = sizes[k][0], H = sizes[k][1];
                const size_t n = (size_t)W * H;
                uint8_t *mask = malloc(n), *st = malloc(n), *tmp = malloc(n), *one = malloc(n);
                for (size_t i = 0; i < n; i++) mask[i] = (uint8_t)((i * 7 + k) % 11 == 0);
                const int walls = (int)(k & 1);
                const double f = (k % 3 == 0) ? 0.0 : 0.0155;
                const uint64_t seed = 1000u + (uint64_t)id;
                expect(fhpo_init(W, H, seed, 0.35, (k & 2) ? mask : NULL, walls, st) == 0, "init", id);
                memcpy(one, st, n);
                int64_t swaps = 0, s1 = 0;
                expect(fhpo_run_rules(st, tmp, W, H, 3, 9, seed, f, chir, rules, 2, &swaps) == 0,
                       "run", id);
                for (uint64_t t = 3; t < 12; t++) {  /* the same steps one at a time, one thread */
                    const int64_t r = fhpo_step_rules(one, tmp, W, H, t, seed, f, chir, rules, 1);
                    expect(r >= 0, "step", id);
                    s1 += r;
                    memcpy(one, tmp, n);
                }
                expect(memcmp(one, st, n) == 0 && s1 == swaps, "run differs from single steps", id);
                int64_t g[11];
                fhpo_observe_global(st, W, H, g);
                int64_t *rows = malloc(sizeof(int64_t) * 3 * H), rsum = 0;
                fhpo_observe_rows(st, W, H, rows);
                for (uint32_t y = 0; y < H; y++) rsum += rows[3 * y];
                expect(rsum == g[0], "row sums", id);
                int64_t bsum = 0;
                for (size_t b = 0; b < sizeof blocks / sizeof blocks[0]; b++) {
                    const uint32_t bb = blocks[b];
                    const size_t nb = (size_t)((H + bb - 1) / bb) * ((W + bb - 1) / bb) * 3;
                    int32_t *out = malloc(sizeof(int32_t) * nb);
                    expect(fhpo_observe_blocks(st, W, H, bb, out) == 0, "blocks", id);
                    int64_t m = 0;
                    for (size_t i = 0; i < nb; i += 3) m += out[i];
                    expect(m == g[0], "block sums", id);
                    bsum += m;
                    free(out);
                }
                if (fhpo_step_rules(st, tmp, W, H, 0, seed, 0.5, chir, rules, 1) != -1)
                    expect(0, "force rate above 1/64 accepted", id);
                printf("case %d %016llx %lld %lld %lld %lld %lld %lld\n", id,
                       (unsigned long long)fhpo_digest(st, W, H), (long long)g[0], (long long)g[1],
                       (long long)g[2], (long long)swaps, (long long)bsum, (long long)rsum);
                free(rows);
                free(mask);
                free(st);
                free(tmp);
                free(one);
            }
        }
    }
    (void)fhpo_hash(~0ull, ~0ull);
    if (fails) return 1;
    printf("OK\n");
    return 0;
}
