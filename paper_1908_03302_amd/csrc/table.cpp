// Host tabulation of the detour function h(R) from a sampled pulse.
//
// h(R) = int_0^inf w^3 S(w) sin(w R/c0) dw / int_0^inf w^2 S(w) dw, S = |F|^2,
// the frequency-domain kernel of Sec. II-C (eq. Kernel_freq) without the
// geometric factor A.  F is the discrete-time Fourier transform of the pulse
// samples; the integrals are uniform trapezoid sums whose node spacing keeps
// the oscillatory integrand free of aliasing up to the largest detour needed.
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"

namespace fftt {

namespace {

// |sum_k f_k exp(-i w k dt) dt|^2 by a rotating phasor (recurrence), with
// the phasor re-seeded from cos/sin every 64 samples to bound drift.
double energy_spectrum(const double* f, int64_t nt, double dt, double w) {
    double re = 0.0, im = 0.0;
    const double c1 = std::cos(w * dt), s1 = std::sin(w * dt);
    double c = 1.0, s = 0.0;
    for (int64_t k = 0; k < nt; ++k) {
        if ((k & 63) == 0) {
            c = std::cos(w * dt * (double)k);
            s = std::sin(w * dt * (double)k);
        }
        re += f[k] * c;
        im -= f[k] * s;
        const double cn = c * c1 - s * s1;
        s = s * c1 + c * s1;
        c = cn;
    }
    return (re * re + im * im) * dt * dt;
}

}  // namespace

int build_table_from_pulse(double c0, const double* f, int64_t nt, double dt, int64_t n,
                           double r_max, double* h_out, double* r_max_out, std::string* err) {
    if (!(c0 > 0) || !std::isfinite(c0) || nt < 2 || !(dt > 0) || !std::isfinite(dt) || n < 2 ||
        n > kMaxTable || !f || !h_out) {
        *err = "build_table_from_pulse: bad argument";
        return -1;
    }
    for (int64_t k = 0; k < nt; ++k)
        if (!std::isfinite(f[k])) {
            *err = "build_table_from_pulse: non-finite pulse sample";
            return -1;
        }
    // 1. Band: scan w^3 S(w) up to the Nyquist frequency.
    const int scan = 8192;
    const double w_nyq = M_PI / dt;
    std::vector<double> g(scan + 1);
    double gmax = 0.0;
    for (int i = 0; i <= scan; ++i) {
        const double w = w_nyq * i / scan;
        g[i] = w * w * w * energy_spectrum(f, nt, dt, w);
        gmax = std::fmax(gmax, g[i]);
    }
    if (!(gmax > 0)) {
        *err = "build_table_from_pulse: pulse has no energy";
        return -1;
    }
    int last = 0;
    for (int i = 0; i <= scan; ++i)
        if (g[i] > 1e-24 * gmax) last = i;
    const double w_top = std::fmin(w_nyq, 1.25 * w_nyq * (last + 1) / scan);

    // 2. Nodes: spacing pi / tau_span with tau_span covering the largest
    //    detour (over c0) plus the pulse length, so sin(w tau) is resolved.
    const double duration = dt * (double)nt;
    const double tau_hi = (r_max > 0 ? r_max / c0 : 2.0 * duration) + duration;
    const double dw = M_PI / tau_hi;
    const int64_t nw = std::max<int64_t>(128, (int64_t)std::ceil(w_top / dw) + 1);
    const double step = w_top / (double)(nw - 1);
    std::vector<double> a(nw), b(nw);
    double den = 0.0;
    for (int64_t m = 0; m < nw; ++m) {
        const double w = step * (double)m;
        const double S = energy_spectrum(f, nt, dt, w);
        const double q = (m == 0 || m == nw - 1) ? 0.5 : 1.0;
        a[m] = q * w * w * w * S;
        den += q * w * w * S;
        b[m] = w / c0;
    }
    for (int64_t m = 0; m < nw; ++m) a[m] /= den;
    auto h_at = [&](double R) {
        double acc = 0.0;
        for (int64_t m = 0; m < nw; ++m) acc += a[m] * std::sin(b[m] * R);
        return acc;
    };

    // 3. Radius: smallest R beyond which |h| stays below 1e-7 max|h|.
    if (!(r_max > 0)) {
        const double R_hi = c0 * 2.0 * duration;
        const int nr = 20000;
        std::vector<double> hv(nr + 1);
        double hm = 0.0;
        for (int i = 0; i <= nr; ++i) {
            hv[i] = h_at(R_hi * i / nr);
            hm = std::fmax(hm, std::fabs(hv[i]));
        }
        int lastbig = 0;
        for (int i = 0; i <= nr; ++i)
            if (std::fabs(hv[i]) >= 1e-7 * hm) lastbig = i;
        r_max = R_hi * (lastbig + 1) / nr;
    }
    for (int64_t k = 0; k < n; ++k) h_out[k] = h_at(r_max * (double)k / (double)(n - 1));
    if (r_max_out) *r_max_out = r_max;
    return 0;
}

// Sine series of the same function (the paper's stored representation of
// eq. Kernel_freq, Sec. II-C): the two frequency integrals as trapezoid sums
// over uniform nodes w_m = m dw, m = 1..n (the node w = 0 contributes
// nothing), so h(R) = sum_m a_m sin(m beta R) with beta = dw / c0 and
// a_m = w_m^3 S(w_m) / sum_k w_k^2 S(w_k).  Both integrands are even in w,
// so the sums converge spectrally once their top node is past the band and
// the spacing is fine enough: the sum is periodic in R with period
// 2 pi c0 / dw, chosen as 2.5 r_max, which keeps the first alias of h at
// R >= 1.5 r_max, where h is negligible.  The band ends at the last
// frequency where w^3 S exceeds tol times its maximum.
int build_series_from_pulse(double c0, const double* f, int64_t nt, double dt, double r_max,
                            double tol, int32_t max_terms, double* a_out, int32_t* n_out,
                            double* beta_out, std::string* err) {
    if (!(c0 > 0) || !std::isfinite(c0) || nt < 2 || !(dt > 0) || !std::isfinite(dt) ||
        !(r_max > 0) || !std::isfinite(r_max) || !(tol > 0 && tol < 1) || max_terms < 1 || !f ||
        !a_out || !n_out || !beta_out) {
        *err = "build_series_from_pulse: bad argument";
        return -1;
    }
    for (int64_t k = 0; k < nt; ++k)
        if (!std::isfinite(f[k])) {
            *err = "build_series_from_pulse: non-finite pulse sample";
            return -1;
        }
    const int scan = 8192;
    const double w_nyq = M_PI / dt;
    std::vector<double> g(scan + 1);
    double gmax = 0.0;
    for (int i = 0; i <= scan; ++i) {
        const double w = w_nyq * i / scan;
        g[i] = w * w * w * energy_spectrum(f, nt, dt, w);
        gmax = std::fmax(gmax, g[i]);
    }
    if (!(gmax > 0)) {
        *err = "build_series_from_pulse: pulse has no energy";
        return -1;
    }
    int last = 0;
    for (int i = 0; i <= scan; ++i)
        if (g[i] > tol * gmax) last = i;
    const double w_top = w_nyq * std::fmin(1.0, (double)(last + 1) / scan);
    const double dw = 2.0 * M_PI * c0 / (2.5 * r_max);
    const int64_t n = (int64_t)std::ceil(w_top / dw);
    if (n > max_terms) {
        *err = "build_series_from_pulse: the band needs " + std::to_string(n) + " terms";
        return -1;
    }
    double den = 0.0;
    for (int64_t m = 1; m <= n; ++m) {
        const double w = dw * (double)m;
        const double S = energy_spectrum(f, nt, dt, w);
        a_out[m - 1] = w * w * w * S;
        den += w * w * S;
    }
    for (int64_t m = 0; m < n; ++m) a_out[m] /= den;
    *n_out = (int32_t)n;
    *beta_out = dw / c0;
    return 0;
}

}  // namespace fftt
