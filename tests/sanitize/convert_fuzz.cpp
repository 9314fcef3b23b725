// Converter fuzz under AddressSanitizer and UndefinedBehaviorSanitizer (host code only): random CSR
// matrices of many shapes and densities, every value type, aggregation and load-balance mode, format
// thresholds, work-range sizes and thread counts; convert, info, export, and the round trip checked
// (structure always, FP64 value bits too).  Built with g++ by tests/test_sanitize.py.
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <vector>
#include <algorithm>
#include "cb_host.h"
namespace cbh { void set_last_error(const std::string &) {} }
static cb_options_t defaults() {
    cb_options_t o{}; o.struct_size = sizeof(o); o.value_type = CB_VALUE_F64; o.col_agg = -1; o.th0 = 0.15;
    o.th1 = 32; o.th2 = 128; o.quantum_tiles = 8; o.lb_mode = CB_LB_CONTIGUOUS; o.host_threads = 0; o.wave_nnz = 0;
    o.row_reduce = -1; o.vector_f64 = 0; o.spmv_kernel = -1; return o;
}
int main(int argc, char **argv) {
    const int iters = argc > 1 ? atoi(argv[1]) : 300;
    std::mt19937_64 rng(12345);
    int fails = 0;
    for (int it = 0; it < iters; ++it) {
        const int64_t m = rng() % 300, n = rng() % 300 + (rng() % 4 == 0 ? 2000 : 0);
        const int mode = rng() % 4;
        std::vector<int64_t> rp(m + 1, 0);
        std::vector<int32_t> ci;
        std::vector<double> va;
        for (int64_t r = 0; r < m; ++r) {
            int64_t len = 0;
            if (n > 0) {
                if (mode == 0) len = rng() % std::min<int64_t>(n, 8);
                else if (mode == 1) len = rng() % 3 == 0 ? std::min<int64_t>(n, rng() % 200) : rng() % 4;
                else if (mode == 2) len = std::min<int64_t>(n, 16 + rng() % 16);  // dense-ish tiles
                else len = (r % 17 == 0) ? std::min<int64_t>(n, 300) : rng() % 3;
            }
            std::vector<int32_t> cols;
            if (mode == 2) { int64_t b = (r / 16) * 16 % std::max<int64_t>(n, 1); for (int64_t c = b; c < std::min(n, b + len); ++c) cols.push_back((int32_t)c); }
            else { std::vector<int32_t> all; for (int64_t k = 0; k < len; ++k) all.push_back((int32_t)(rng() % n)); std::sort(all.begin(), all.end()); all.erase(std::unique(all.begin(), all.end()), all.end()); cols = all; }
            for (int32_t c : cols) { ci.push_back(c); va.push_back((double)(int64_t)(rng() % 2001 - 1000) / 7.0); }
            rp[r + 1] = (int64_t)ci.size();
        }
        const int64_t nnz = (int64_t)ci.size();
        cb_options_t o = defaults();
        o.value_type = (cb_value_t)(rng() % 3);
        o.col_agg = (int)(rng() % 3) - 1;
        o.lb_mode = (int)(rng() % 3);
        const int th = rng() % 3;
        if (th == 1) { o.th1 = 16; o.th2 = 64; } else if (th == 2) { o.th1 = 257; o.th2 = 257; }
        if (rng() % 2) o.wave_nnz = 1 + rng() % 200;
        o.host_threads = 1 + rng() % 4;
        o.row_reduce = (int)(rng() % 6) - 1;
        cbh::HostStructure s;
        std::string err;
        cb_status_t st = cbh::convert(m, n, nnz, rp.data(), ci.data(), va.empty() ? nullptr : va.data(), o, s, err);
        if (st != CB_SUCCESS) { printf("it %d convert failed: %s\n", it, err.c_str()); ++fails; continue; }
        cb_info_t info{}; info.struct_size = sizeof(info);
        cbh::fill_info(s, info);
        (void)cbh::spmv_bytes(s);
        std::vector<int64_t> rp2(m + 1);
        std::vector<int32_t> ci2(nnz + 1);
        std::vector<double> va2(nnz + 1);
        st = cbh::export_csr(s, rp2.data(), ci2.data(), va2.data(), err);
        if (st != CB_SUCCESS) { printf("it %d export failed: %s\n", it, err.c_str()); ++fails; continue; }
        bool ok = std::equal(rp.begin(), rp.end(), rp2.begin()) && std::equal(ci.begin(), ci.end(), ci2.begin());
        if (o.value_type == CB_VALUE_F64) ok = ok && (nnz == 0 || memcmp(va.data(), va2.data(), 8 * nnz) == 0);
        if (!ok) { printf("it %d round trip mismatch (m %lld n %lld nnz %lld vt %d)\n", it, (long long)m, (long long)n, (long long)nnz, o.value_type); ++fails; }
    }
    printf("iterations %d failures %d\n", iters, fails);
    return fails ? 1 : 0;
}
