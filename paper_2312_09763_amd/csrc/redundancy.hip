// Host side of the redundancy-aware product (App. A): baseline redundancy
// groups and the sub-matrix heuristic.  Plain C++ on the host, deterministic.
//
// Baselines are the pairs (i, j), i <= j, in lexicographic order.  Two are
// redundant when their antennas carry the same beams and their vectors
// x_i - x_j agree to within tol in every component; a pair joins the earliest
// group whose representative it matches, else it founds a group (so the
// representative is the group's first pair).  The match search looks at the
// 27 cells of side 2 tol around the vector, which hold every representative
// within tol (with a margin for the rounding of the cell index), and keeps
// the smallest group id: the same groups as comparing
// against every representative in creation order.
//
// The heuristic follows App. A's steps: order the first antennas of the
// pairs by multiplicity (descending, ties by index), then place N_sub - 1
// cuts, each after the last prefix whose density (pairs covered / sub-matrix
// size) is still >= tau, keeping one antenna for every later sub-matrix; if
// the last sub-matrix is not denser than tau, lower tau (tau_k = 1 - 0.01 k)
// and place the cuts again.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <tuple>
#include <vector>

#include "internal.h"
#include "matvis.h"

namespace mv {
namespace red {

int64_t groups(const double *antpos, const int32_t *beam_idx, int n_ant, double tol, int32_t *group, int32_t *rep_a,
               int32_t *rep_b) {
    typedef std::tuple<int32_t, int32_t, int64_t, int64_t, int64_t> Key;
    std::map<Key, std::vector<int32_t>> cells;  // cell -> groups whose representative lies in it
    std::vector<double> rv;                     // representative vectors, 3 per group
    std::vector<int32_t> rb;                    // representative beams, 2 per group
    int64_t n_groups = 0, p = 0;
    for (int i = 0; i < n_ant; i++)
        for (int j = i; j < n_ant; j++, p++) {
            const int32_t bi = beam_idx ? beam_idx[i] : 0, bj = beam_idx ? beam_idx[j] : 0;
            double b[3];
            int64_t q[3];
            for (int d = 0; d < 3; d++) {
                b[d] = antpos[3 * i + d] - antpos[3 * j + d];
                q[d] = (int64_t)std::floor(b[d] / (2.0 * tol));  // cells of 2 tol: a match is within one cell
            }
            int64_t found = -1;
            for (int dx = -1; dx <= 1; dx++)
                for (int dy = -1; dy <= 1; dy++)
                    for (int dz = -1; dz <= 1; dz++) {
                        auto it = cells.find(Key(bi, bj, q[0] + dx, q[1] + dy, q[2] + dz));
                        if (it == cells.end()) continue;
                        for (int32_t g : it->second) {
                            if (found >= 0 && g >= found) break;  // groups are listed in creation order
                            if (rb[2 * g] != bi || rb[2 * g + 1] != bj) continue;
                            bool ok = true;
                            for (int d = 0; d < 3; d++)
                                if (!(std::fabs(b[d] - rv[3 * g + d]) <= tol)) ok = false;
                            if (ok) found = g;
                        }
                    }
            if (found < 0) {
                found = n_groups++;
                rep_a[found] = i;
                rep_b[found] = j;
                rv.insert(rv.end(), b, b + 3);
                rb.push_back(bi);
                rb.push_back(bj);
                cells[Key(bi, bj, q[0], q[1], q[2])].push_back((int32_t)found);
            }
            group[p] = (int32_t)found;
        }
    return n_groups;
}

Plan plan(const int32_t *pa, const int32_t *pb, int n_pair, int n_ant, int n_sub) {
    Plan P;
    std::vector<int64_t> mult(n_ant, 0);
    std::vector<std::vector<int32_t>> seconds(n_ant);
    for (int u = 0; u < n_pair; u++) {
        mult[pa[u]]++;
        seconds[pa[u]].push_back(pb[u]);
    }
    std::vector<int> alpha;
    for (int a = 0; a < n_ant; a++)
        if (mult[a] > 0) alpha.push_back(a);
    std::stable_sort(alpha.begin(), alpha.end(), [&](int x, int y) { return mult[x] > mult[y]; });
    const int na = (int)alpha.size();
    n_sub = std::max(1, std::min(n_sub, na));
    std::vector<int> mark(n_ant, -1);  // stamp of the prefix scan that last added the antenna to beta
    int stamp = 0;
    std::vector<int> sizes;
    for (int k = 0;; k++) {
        const double tau = 1.0 - (double)k * 0.01;
        sizes.clear();
        int start = 0;
        for (int x = 0; x < n_sub - 1; x++) {
            const int max_n = na - start - (n_sub - 1 - x);
            int best = 1;
            int64_t cnt = 0, nbeta = 0;
            stamp++;
            for (int n = 1; n <= max_n; n++) {
                const int a = alpha[start + n - 1];
                cnt += mult[a];
                for (int b : seconds[a])
                    if (mark[b] != stamp) {
                        mark[b] = stamp;
                        nbeta++;
                    }
                const double d = (double)cnt / (double)((int64_t)n * nbeta);
                if (d >= tau)
                    best = n;
                else
                    break;
            }
            sizes.push_back(best);
            start += best;
        }
        sizes.push_back(na - start);
        int64_t cnt = 0, nbeta = 0;
        stamp++;
        for (int n = start; n < na; n++) {
            cnt += mult[alpha[n]];
            for (int b : seconds[alpha[n]])
                if (mark[b] != stamp) {
                    mark[b] = stamp;
                    nbeta++;
                }
        }
        const double d_last = (double)cnt / (double)((int64_t)sizes.back() * nbeta);
        if (d_last > tau || tau <= 0.0) break;
    }
    P.alpha = alpha;
    P.sizes = sizes;
    int start = 0;
    for (int n : sizes) {
        std::vector<int> A(alpha.begin() + start, alpha.begin() + start + n), B;
        int64_t cnt = 0;
        stamp++;
        for (int a : A) {
            cnt += mult[a];
            for (int b : seconds[a])
                if (mark[b] != stamp) {
                    mark[b] = stamp;
                    B.push_back(b);
                }
        }
        std::sort(B.begin(), B.end());
        P.density.push_back((double)cnt / (double)((int64_t)A.size() * B.size()));
        P.A.push_back(A);
        P.B.push_back(B);
        start += n;
    }
    return P;
}

}  // namespace red
}  // namespace mv

using namespace mv;

extern "C" {

matvis_status matvis_redundant_groups(const double *antpos, const int32_t *beam_idx, int32_t n_ant, double tol_m,
                                      int32_t *group, int32_t *rep_a, int32_t *rep_b, int32_t *n_unique) {
    if (!antpos || !group || !rep_a || !rep_b || !n_unique || n_ant <= 0 || n_ant > 8192) return MATVIS_EINVAL;
    if (!(tol_m > 0.0) || !std::isfinite(tol_m)) return MATVIS_EINVAL;
    for (int i = 0; i < 3 * n_ant; i++)
        if (!std::isfinite(antpos[i])) return MATVIS_EINVAL;
    *n_unique = (int32_t)red::groups(antpos, beam_idx, n_ant, tol_m, group, rep_a, rep_b);
    return MATVIS_OK;
}

matvis_status matvis_submatrix_plan(const int32_t *pair_a, const int32_t *pair_b, int32_t n_pair, int32_t n_ant,
                                    int32_t n_sub, int32_t *alpha, int32_t *sizes, double *density, int32_t *n_alpha,
                                    int32_t *n_sub_out) {
    if (!pair_a || !pair_b || !alpha || !sizes || !density || !n_alpha || !n_sub_out) return MATVIS_EINVAL;
    if (n_pair <= 0 || n_ant <= 0 || n_sub <= 0) return MATVIS_EINVAL;
    for (int u = 0; u < n_pair; u++)
        if (pair_a[u] < 0 || pair_a[u] >= n_ant || pair_b[u] < 0 || pair_b[u] >= n_ant) return MATVIS_EINVAL;
    red::Plan P = red::plan(pair_a, pair_b, n_pair, n_ant, n_sub);
    std::copy(P.alpha.begin(), P.alpha.end(), alpha);
    std::copy(P.sizes.begin(), P.sizes.end(), sizes);
    std::copy(P.density.begin(), P.density.end(), density);
    *n_alpha = (int32_t)P.alpha.size();
    *n_sub_out = (int32_t)P.sizes.size();
    return MATVIS_OK;
}

}  // extern "C"
