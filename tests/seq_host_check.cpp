// Host check of the residual kernels' segment positions (es_seq.h, compiled for
// the CPU): the line, along-coordinate and transverse coordinates that seq_base /
// seq_at derive by carries must equal those of a plain floor division of the
// position within its sequence (line = ls x sequence line + j), for every base and
// lane offset a segment can have, on lines of 1..70 nodes with 3 or 4 ghost layers
// and 1, 2 or 4 sequences.  Exit status 0 when all agree.
#include <cstdio>
#define __device__
#define __host__
#define __forceinline__ inline
#include "es_seq.h"
using namespace es;

int main() {
    long long bad = 0, checks = 0;
    for (int n = 1; n <= 70; ++n)
        for (int ng = 3; ng <= 4; ++ng)
            for (int nf = 1; nf <= 9; nf += 4)
            for (int ls = 1; ls <= 4; ls *= 2)
            for (int j = 0; j < ls; ++j) {
                const int pl = n + 2 * ng;
                for (long long base = -6; base < 3 * pl + 5; ++base) {
                    const SeqBase b = seq_base(base, pl, ng, nf, ls, j);
                    for (int q = 0; q < 70; ++q) {
                        long long lid;
                        int s, fa, fb;
                        seq_at(b, q, true, pl, ng, nf, ls, j, lid, s, fa, fb);
                        const long long f = base + q;
                        const long long em = f >= 0 ? f / pl : -((-f + pl - 1) / pl);
                        const long long el = em * ls + j;
                        const int es = (int)(f - em * pl) - ng;
                        ++checks;
                        bool ok = lid == el && s == es;
                        if (ok && lid >= 0) ok = fa == (int)(lid % nf) && fb == (int)(lid / nf);
                        if (!ok) {
                            if (bad < 5)
                                printf("mismatch n=%d ng=%d nf=%d base=%lld q=%d: (%lld, %d, %d, %d)\n", n, ng, nf,
                                       base, q, lid, s, fa, fb);
                            ++bad;
                        }
                    }
                }
            }
    // aligned layout: segment w of a sequence starts nsl segments per line, lane 0 at
    // along-coordinate (w mod nsl) seg - halo - ng of line w / nsl, without wrapping
    for (int nsl = 1; nsl <= 4; ++nsl)
        for (int seg = 54; seg <= 61; seg += 7)
            for (int halo = 0; halo <= 5; halo += 5)
                for (int nf = 1; nf <= 9; nf += 4)
                    for (int ls = 1; ls <= 4; ls *= 2)
                        for (int j = 0; j < ls; ++j)
                            for (long long w = 0; w < 40; ++w) {
                                const int ng = 3, pl = nsl * seg;
                                const SeqBase b = seq_base_aligned(w, nsl, seg, halo, ng, nf, ls, j);
                                for (int q = 0; q < 70; ++q) {
                                    long long lid;
                                    int s, fa, fb;
                                    seq_at(b, q, false, pl, ng, nf, ls, j, lid, s, fa, fb);
                                    const long long el = (w / nsl) * ls + j;
                                    const int es = (int)(w % nsl) * seg - halo - ng + q;
                                    ++checks;
                                    bool ok = lid == el && s == es && fa == (int)(el % nf) && fb == (int)(el / nf);
                                    if (!ok) {
                                        if (bad < 5) printf("aligned mismatch nsl=%d w=%lld q=%d\n", nsl, w, q);
                                        ++bad;
                                    }
                                }
                            }
    // the layout rule: 128-node lines (p = 3) take the flat layout, 400-node lines
    // the aligned one
    ++checks;
    if (!seq_flat(128, 134, 61, 0.875) || seq_flat(400, 406, 61, 0.875)) {
        printf("layout rule mismatch\n");
        ++bad;
    }
    printf("%lld positions, %lld mismatches\n", checks, bad);
    return bad != 0;
}
