// Line positions of the residual kernels' segments (device code; also compiled for
// the host by tests/seq_host_check.cpp).
#pragma once

namespace es {

// Positions along the lines of one axis for the residual kernels' segments.  The
// lines are dealt to ls sequences, sequence j holding lines j, j + ls, j + 2 ls, ...,
// so that the ls wavefronts of a block, one per sequence at the same offset, work on
// ls adjacent lines at the same along-coordinates (their strided loads share cache
// lines).  Within a sequence the segments are laid out in one of two ways:
// * flat: the lines' padded node sequences (pl = n + 2 ng nodes each, the ng ghost
//   nodes first) laid end to end, so that a segment may run from one line into the
//   next and no wavefront is left nearly idle at a line's end;
// * aligned: nsl segments per line, the first at the line's start (positions past
//   the line's padded end are not used).
// A wavefront's lanes hold consecutive positions base + q; the line and
// along-coordinate of each follow from those of base (one division per wavefront)
// by short carries, so no lane divides.  nf is the number of lines along the faster
// transverse axis.
struct SeqBase {
    long long m;     // line of position base within the sequence (-1 before the first)
    int s;           // along-coordinate of base
    int fa, fb;      // transverse coordinates of line max(m, 0) of the sequence
};

__device__ __forceinline__ void seq_line_coords(SeqBase& b, int nf, int ls, int j) {
    const long long lid = (b.m >= 0 ? b.m : 0) * ls + j;
    b.fa = (int)(lid % nf);
    b.fb = (int)(lid / nf);
}

// flat layout: base is a position of the end-to-end sequence
__device__ __forceinline__ SeqBase seq_base(long long base, int pl, int ng, int nf, int ls, int j) {
    SeqBase b;
    b.m = base >= 0 ? base / pl : -((-base + pl - 1) / pl);
    b.s = (int)(base - b.m * pl) - ng;
    seq_line_coords(b, nf, ls, j);
    return b;
}

// aligned layout: segment w of the sequence (nsl per line, seg positions apart),
// lane 0 at along-coordinate k seg - halo - ng of its line, k = w mod nsl
__device__ __forceinline__ SeqBase seq_base_aligned(long long w, int nsl, int seg, int halo, int ng, int nf, int ls,
                                                    int j) {
    SeqBase b;
    b.m = w / nsl;
    b.s = (int)(w - b.m * nsl) * seg - halo - ng;
    seq_line_coords(b, nf, ls, j);
    return b;
}

// line (lid, negative before the first), along-coordinate (s) and transverse
// coordinates (fa, fb) of position base + q of sequence j; lid may pass the last
// line and, aligned, s the line's padded end (the caller checks both)
__device__ __forceinline__ void seq_at(const SeqBase& b, int q, bool flat, int pl, int ng, int nf, int ls, int j,
                                       long long& lid, int& s, int& fa, int& fb) {
    long long m = b.m;
    s = b.s + q;
    if (flat) {
        while (s >= pl - ng) {
            s -= pl;
            ++m;
        }
    }
    lid = m * ls + j;
    fa = b.fa;
    fb = b.fb;
    for (long long d = b.m < 0 ? m : m - b.m; d > 0; --d) {
        fa += ls;
        while (fa >= nf) { fa -= nf; ++fb; }
    }
}

// whether the flat layout is used: the positions of a line that segments must
// cover (cover; the aligned layout takes ceil(cover / seg) segments per line) against
// the padded line length pl of the flat one; flat when it needs at most `ratio` of
// the aligned layout's wavefronts (a flat segment costs somewhat more: it may hold
// two lines)
__host__ __device__ inline bool seq_flat(int cover, int pl, int seg, double ratio) {
    const int nsl = (cover + seg - 1) / seg;
    return (double)pl <= ratio * (double)nsl * (double)seg;
}

}  // namespace es
