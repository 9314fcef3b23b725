// Converter check of the streaming kernel's 32-bit range offsets (host code only): a work range whose
// payload would span more bytes than the limit is refused with CB_ERROR_INVALID_VALUE and a message,
// not truncated into the int32 batch records.  The real limit (2 GiB) needs a matrix of about 240 M
// non-zeros in one range, so this program converts a small 3D block matrix against a 64 KB limit:
// automatic ranges pass, one range holding the whole matrix is refused.  Built by tests/test_sanitize.py.
#include <cstdio>
#include <string>
#include <vector>
#include "cb_host.h"
namespace cbh { void set_last_error(const std::string &) {} }
int main() {
    // 7-point adjacency on a 12^3 grid, one unknown per node
    const int side = 12, N = side * side * side;
    std::vector<int64_t> rp(1, 0);
    std::vector<int32_t> ci;
    std::vector<double> va;
    for (int k = 0; k < side; ++k)
        for (int j = 0; j < side; ++j)
            for (int i = 0; i < side; ++i) {
                const int r = i + side * (j + side * k);
                const int nb[7] = {k > 0 ? r - side * side : -1, j > 0 ? r - side : -1, i > 0 ? r - 1 : -1, r,
                                   i + 1 < side ? r + 1 : -1, j + 1 < side ? r + side : -1,
                                   k + 1 < side ? r + side * side : -1};
                for (int c : nb)
                    if (c >= 0) { ci.push_back(c); va.push_back(c == r ? 6.0 : -1.0); }
                rp.push_back((int64_t)ci.size());
            }
    cb_options_t o{};
    o.struct_size = sizeof(o); o.value_type = CB_VALUE_F64; o.col_agg = -1; o.th0 = 0.15; o.th1 = 32; o.th2 = 128;
    o.quantum_tiles = 8; o.host_threads = 1; o.row_reduce = -1; o.vector_f64 = 0; o.spmv_kernel = -1;
    const int64_t limit = 64 << 10;
    int bad = 0;
    for (int lb : {CB_LB_CONTIGUOUS, CB_LB_NONE}) {
        o.lb_mode = lb;
        std::string err;
        cbh::HostStructure s;
        o.wave_nnz = 0;
        cb_status_t st = cbh::convert(N, N, (int64_t)ci.size(), rp.data(), ci.data(), va.data(), o, s, err, limit);
        std::printf("lb %d automatic ranges: status %d (%s), payload %lld bytes, %lld ranges\n", lb, (int)st,
                    err.c_str(), (long long)s.payload_bytes, (long long)s.nwaves);
        if (st != CB_SUCCESS || s.payload_bytes <= limit) bad = 1;
        cbh::HostStructure s2;
        err.clear();
        o.wave_nnz = (int64_t)ci.size() * 4;
        st = cbh::convert(N, N, (int64_t)ci.size(), rp.data(), ci.data(), va.data(), o, s2, err, limit);
        std::printf("lb %d one range: status %d (%s)\n", lb, (int)st, err.c_str());
        if (st != CB_ERROR_INVALID_VALUE || err.find("wave_nnz too large") == std::string::npos) bad = 1;
        // the default limit accepts the same request
        cbh::HostStructure s3;
        err.clear();
        st = cbh::convert(N, N, (int64_t)ci.size(), rp.data(), ci.data(), va.data(), o, s3, err);
        std::printf("lb %d one range, 2 GiB limit: status %d\n", lb, (int)st);
        if (st != CB_SUCCESS || s3.nwaves != 1) bad = 1;
    }
    std::printf(bad ? "FAILED\n" : "ok\n");
    return bad;
}
