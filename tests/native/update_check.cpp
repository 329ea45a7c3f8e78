// Host build of the GPU library's per-word update (fhp_device.h) checked
// against the CPU oracle's collision tables of the three rule sets, for every
// 7-bit state, both chiralities, fluid and solid nodes, and the forcing swap.  Test code only:
// it links the oracle and includes the library header side by side.
#include <stdio.h>

#include "../../paper_1208_2428_amd/csrc/fhp_device.h"
extern "C" {
#include "../../oracle/fhp_oracle.h"
}

// Every (state, chirality) pair of rule set RULES, on fluid and solid nodes.
template <int RULES>
int check_rules(int oracle_rules) {
    uint8_t table[2][128];
    if (fhpo_rule_table(oracle_rules, 0, table[0]) || fhpo_rule_table(oracle_rules, 1, table[1])) {
        printf("rule set %d unknown to the oracle\n", oracle_rules);
        return 1;
    }
    int bad = 0;
    // 256 (state, chirality) combinations in four words of 64 nodes
    for (int k = 0; k < 4; k++) {
        uint64_t a[7] = {0}, chi = 0;
        for (int b = 0; b < 64; b++) {
            const int combo = k * 64 + b, s = combo & 127;
            for (int c = 0; c < 7; c++)
                if ((s >> c) & 1) a[c] |= 1ull << b;
            if (combo >> 7) chi |= 1ull << b;
        }
        for (int solid = 0; solid < 2; solid++) {
            uint64_t o[7];
            fhp::update<RULES>(a, solid ? ~0ull : 0ull, chi, 0, o);
            for (int b = 0; b < 64; b++) {
                const int combo = k * 64 + b, s = combo & 127;
                int got = 0;
                for (int c = 0; c < 7; c++) got |= (int)((o[c] >> b) & 1) << c;
                int want;
                if (solid) {  // bounce-back c_i -> c_{i+3}, rest kept
                    want = s & 64;
                    for (int i = 0; i < 6; i++) want |= ((s >> ((i + 3) % 6)) & 1) << i;
                } else {
                    want = table[combo >> 7][s];
                }
                if (got != want) {
                    if (bad < 10)
                        printf("rules %d state %d chi %d solid %d: got %d want %d\n", oracle_rules,
                               s, combo >> 7, solid, got, want);
                    bad++;
                }
            }
        }
    }
    // forcing: lone W-movers (no collision in any rule set); coin on node 17
    // flips it to E on a fluid node, and does nothing on a solid node (which
    // bounces it back)
    {
        uint64_t a[7] = {0}, o[7];
        a[5] = ~0ull;
        fhp::update<RULES>(a, 0, 0, 1ull << 17, o);
        if (o[5] != ~(1ull << 17) || o[2] != (1ull << 17)) bad++, printf("forcing on fluid\n");
        fhp::update<RULES>(a, 1ull << 17, 0, 1ull << 17, o);
        if (o[2] != (1ull << 17) || o[5] != ~(1ull << 17)) bad++, printf("forcing on solid\n");
    }
    return bad;
}

int main() {
    int bad = check_rules<fhp::kRulesFHP2>(FHPO_RULES_FHP2);
    bad += check_rules<fhp::kRulesFHP1>(FHPO_RULES_FHP1);
    bad += check_rules<fhp::kRulesFHP3>(FHPO_RULES_FHP3);
    // the hash: SplitMix64 output 1 of state 1234567
    if (fhp::hash64(1234567, 0) != 6457827717110365317ull) bad++, printf("hash\n");
    // split hash = direct hash
    for (uint64_t t = 0; t < 5; t++)
        for (uint64_t y = 0; y < 7; y++)
            for (uint64_t w = 0; w < 9; w++)
                if (fhp::mix64(fhp::word_base(12345, w) + fhp::row_term(t, y)) !=
                    fhp::hash64(12345, fhp::counter(t, y, w)))
                    bad++;
    printf("%s (%d mismatches)\n", bad ? "FAIL" : "OK", bad);
    return bad != 0;
}
