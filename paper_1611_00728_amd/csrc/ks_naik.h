// Sign of a stored Naik matrix relative to its SU(3) part for 12-real storage.
#pragma once

namespace ks {

// Stored Naik slot s at site c (s < 4: W_mu(x); s >= 4: -W_mu(x - 3 mu)^+, mu = s & 3) equals
// c0 * naik_sign(c, s, Nt) * U with U in SU(3), for links that carry the staggered phase
// eta_mu(x) (eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y), eta_3 = (-1)^(x+y+z); eta_mu does
// not depend on x_mu, so the backward link has the phase of x) and -1 on three-links that
// cross the antiperiodic time boundary (forward from t >= Nt - 3, backward from t < 3).
__host__ __device__ inline double naik_sign(const int c[4], int s, int nt)
{
    const int mu = s & 3;
    int e = 0;
    if (mu >= 1) e += c[0];
    if (mu >= 2) e += c[1];
    if (mu >= 3) e += c[2];
    double sg = (e & 1) ? -1.0 : 1.0;
    if (s < 4) {
        if (mu == 3 && c[3] >= nt - 3) sg = -sg;
    } else {
        sg = -sg;
        if (mu == 3 && c[3] < 3) sg = -sg;
    }
    return sg;
}

}  // namespace ks
