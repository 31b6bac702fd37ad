/* Forward echo simulator for seeded point-scatterer phantoms (input generator).
 *
 * For each transmit t, element e, frame f the complex baseband (IQ) record is
 *   iq[t,e,s,f] = sum_k A_k g(ts - tau_k) exp(-j 2 pi fd tau_k) exp(j 2 pi (fc - fd)(ts - tau_k))
 * with ts = t0 + s/fs, g(x) = exp(-x^2 / (2 sigma^2)) truncated at |x| <= trunc*sigma,
 * tau_k = (n_t . x_k)/c + |x_k - p_e|/c  (plane wave crossing the origin at t = 0,
 * spherical return to the element).  This is the physics of the phantom, not a
 * beamformer: it maps scatterers to channel data.
 *
 * The Gaussian and the carrier are advanced sample by sample with exact
 * multiplicative recurrences (two real multiplies and one complex multiply per
 * sample), accumulated in double precision and rounded once to float32.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

void synth_echo(float *iq, int T, int E, int S, int F,
                const double *elem, const double *tx_normal,
                const double *scat, const double *amp, int K,
                double c, double fs, double fc, double fd, double t0,
                double sigma, double trunc_sigmas)
{
    const double two_pi = 6.283185307179586476925286766559;
    const double h = 1.0 / fs;
    const double inv2s2 = 1.0 / (2.0 * sigma * sigma);
    const double q = exp(-h * h / (sigma * sigma));
    const double wr = cos(two_pi * (fc - fd) * h), wi = sin(two_pi * (fc - fd) * h);
    const double half = trunc_sigmas * sigma;
#pragma omp parallel
    {
        double *acc = (double *)malloc(sizeof(double) * 2 * (size_t)S * (size_t)F);
#pragma omp for schedule(dynamic, 1)
        for (long te = 0; te < (long)T * E; ++te) {
            const int t = (int)(te / E), e = (int)(te % E);
            const double ex = elem[3 * e], ey = elem[3 * e + 1], ez = elem[3 * e + 2];
            const double nx = tx_normal[3 * t], ny = tx_normal[3 * t + 1], nz = tx_normal[3 * t + 2];
            memset(acc, 0, sizeof(double) * 2 * (size_t)S * (size_t)F);
            for (int f = 0; f < F; ++f) {
                const double *xs = scat + (size_t)f * K * 3;
                const double *as = amp + (size_t)f * K;
                for (int k = 0; k < K; ++k) {
                    const double x = xs[3 * k], y = xs[3 * k + 1], z = xs[3 * k + 2];
                    const double dx = x - ex, dy = y - ey, dz = z - ez;
                    const double tau = (nx * x + ny * y + nz * z) / c + sqrt(dx * dx + dy * dy + dz * dz) / c;
                    long lo = (long)ceil((tau - half - t0) * fs);
                    long hi = (long)floor((tau + half - t0) * fs);
                    if (lo < 0) lo = 0;
                    if (hi > S - 1) hi = S - 1;
                    if (lo > hi) continue;
                    const double a = t0 + lo * h - tau;           /* ts - tau at s = lo */
                    double g = as[k] * exp(-a * a * inv2s2);       /* amplitude times Gaussian */
                    double r = exp(-(2.0 * a * h + h * h) * inv2s2); /* g[m+1]/g[m] */
                    const double ph = -two_pi * fd * tau + two_pi * (fc - fd) * a;
                    double pr = cos(ph), pi = sin(ph);
                    for (long s = lo; s <= hi; ++s) {
                        double *o = acc + 2 * ((size_t)s * F + f);
                        o[0] += g * pr;
                        o[1] += g * pi;
                        g *= r;
                        r *= q;
                        const double npr = pr * wr - pi * wi;
                        pi = pr * wi + pi * wr;
                        pr = npr;
                    }
                }
            }
            float *dst = iq + 2 * (size_t)te * S * F;
            for (size_t i = 0; i < 2 * (size_t)S * F; ++i) dst[i] = (float)acc[i];
        }
        free(acc);
    }
}
