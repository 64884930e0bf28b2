// Driver for a host build of the table and sine-series builders (table.cpp)
// under AddressSanitizer and UndefinedBehaviorSanitizer.  Not part of the
// library; built and run by the test suite with g++ (host code only).
//
//   table_check <pulses.bin>
//
// pulses.bin: int64 count, then per pulse int64 nt, float64 dt, float64
// r_max, nt float64 samples.  For each pulse: tables of 2, 3, 4096 and 16384
// nodes with the given and with the automatic truncation radius, sine series
// with a loose and a tight tolerance, a term budget too small to succeed,
// and the invalid-argument statuses.  Prints a checksum; exits non-zero on
// an unexpected status or a non-finite value.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "internal.h"

namespace {

double checksum = 0.0;
int bad = 0;

void fold(const char* what, const double* v, int64_t n) {
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(v[i])) {
            std::fprintf(stderr, "%s: non-finite value at %lld\n", what, (long long)i);
            bad = 1;
            return;
        }
        checksum += std::fabs(v[i]) * (double)((i % 5) + 1);
    }
}

void expect(bool ok, const char* what) {
    if (!ok) {
        std::fprintf(stderr, "unexpected status: %s\n", what);
        bad = 1;
    }
}

}  // namespace

int main(int argc, char** argv) {
    if (argc != 2) {
        std::fprintf(stderr, "usage: %s pulses.bin\n", argv[0]);
        return 2;
    }
    FILE* fp = std::fopen(argv[1], "rb");
    if (!fp) {
        std::perror(argv[1]);
        return 2;
    }
    int64_t np = 0;
    if (std::fread(&np, sizeof np, 1, fp) != 1 || np < 1 || np > 16) return 2;
    const double c0 = 1500.0;
    for (int64_t p = 0; p < np; ++p) {
        int64_t nt = 0;
        double dt = 0.0, rm = 0.0;
        if (std::fread(&nt, sizeof nt, 1, fp) != 1 || std::fread(&dt, sizeof dt, 1, fp) != 1 ||
            std::fread(&rm, sizeof rm, 1, fp) != 1 || nt < 1 || nt > (1 << 22))
            return 2;
        std::vector<double> f((size_t)nt);
        if (std::fread(f.data(), sizeof(double), (size_t)nt, fp) != (size_t)nt) return 2;
        std::string err;
        for (int64_t n : {2, 3, 4096, 16384}) {
            std::vector<double> h((size_t)n);
            double r_out = 0.0;
            expect(fftt::build_table_from_pulse(c0, f.data(), nt, dt, n, rm, h.data(), &r_out,
                                                &err) == 0,
                   "table, given r_max");
            fold("table", h.data(), n);
            expect(fftt::build_table_from_pulse(c0, f.data(), nt, dt, n, 0.0, h.data(), &r_out,
                                                &err) == 0,
                   "table, automatic r_max");
            fold("table auto", h.data(), n);
            checksum += r_out;
        }
        {
            std::vector<double> h(8);
            double r_out = 0.0;
            expect(fftt::build_table_from_pulse(c0, f.data(), nt, dt, 1, rm, h.data(), &r_out,
                                                &err) != 0,
                   "table of one node refused");
            expect(fftt::build_table_from_pulse(c0, f.data(), 0, dt, 8, rm, h.data(), &r_out,
                                                &err) != 0,
                   "empty pulse refused");
            expect(fftt::build_table_from_pulse(-c0, f.data(), nt, dt, 8, rm, h.data(), &r_out,
                                                &err) != 0,
                   "negative c0 refused");
            expect(fftt::build_table_from_pulse(c0, f.data(), nt, -dt, 8, rm, h.data(), &r_out,
                                                &err) != 0,
                   "negative dt refused");
        }
        for (double tol : {1e-4, 1e-8}) {
            std::vector<double> a(64);
            int32_t n_terms = 0;
            double beta = 0.0;
            expect(fftt::build_series_from_pulse(c0, f.data(), nt, dt, rm, tol, 64, a.data(),
                                                 &n_terms, &beta, &err) == 0,
                   "series");
            if (n_terms < 1 || n_terms > 64) {
                bad = 1;
                continue;
            }
            fold("series", a.data(), n_terms);
            checksum += beta + n_terms;
        }
        {
            std::vector<double> a(2);
            int32_t n_terms = 0;
            double beta = 0.0;
            expect(fftt::build_series_from_pulse(c0, f.data(), nt, dt, rm, 1e-12, 2, a.data(),
                                                 &n_terms, &beta, &err) != 0,
                   "too few terms refused");
            expect(fftt::build_series_from_pulse(c0, f.data(), nt, dt, -rm, 1e-8, 2, a.data(),
                                                 &n_terms, &beta, &err) != 0,
                   "negative r_max refused");
        }
    }
    std::fclose(fp);
    std::printf("checksum %.17g\n", checksum);
    return bad;
}
