/* Uses the C ABI from C: struct sizes and field offsets as the C compiler lays them out (the Python
 * binding's ctypes mirrors are compared against these), and a host-only conversion with its CSR
 * export, which needs no GPU. */
#include <stddef.h>
#include <stdint.h>
#include <stdio.h>

#include "cbspmv.h"

#define FIELD(T, f) printf("%s.%s %zu\n", #T, #f, offsetof(T, f))
#define SIZE(T) printf("%s %zu\n", #T, sizeof(T))

int main(void) {
    SIZE(cb_options_t);
    FIELD(cb_options_t, th0);
    FIELD(cb_options_t, wave_nnz);
    FIELD(cb_options_t, row_reduce);
    FIELD(cb_options_t, vector_f64);
    FIELD(cb_options_t, spmv_kernel);
    FIELD(cb_options_t, xcd_chunk);
    SIZE(cb_info_t);
    FIELD(cb_info_t, super_sparse_share);
    FIELD(cb_info_t, spmv_bytes);
    FIELD(cb_info_t, convert_seconds);
    FIELD(cb_info_t, nbatches);
    FIELD(cb_info_t, flat_run_mean);
    FIELD(cb_info_t, row_reduce);
    FIELD(cb_info_t, vector_f64);
    FIELD(cb_info_t, spmv_kernel);
    FIELD(cb_info_t, xcd_chunk);
    SIZE(cb_structure_t);
    SIZE(cb_cg_options_t);
    FIELD(cb_cg_options_t, inner_rtol);
    FIELD(cb_cg_options_t, refine_method);
    FIELD(cb_cg_options_t, replace_factor);
    SIZE(cb_cg_result_t);
    FIELD(cb_cg_result_t, rel_residual);
    SIZE(cb_server_options_t);
    FIELD(cb_server_options_t, arena_bytes);
    FIELD(cb_server_options_t, spmm_streams);
    SIZE(cb_request_t);
    FIELD(cb_request_t, alpha);
    FIELD(cb_request_t, in);
    FIELD(cb_request_t, out);
    FIELD(cb_request_t, rtol);
    FIELD(cb_request_t, max_iter);
    SIZE(cb_response_t);
    FIELD(cb_response_t, rel_residual);
    FIELD(cb_response_t, queue_us);
    SIZE(cb_server_stats_t);
    FIELD(cb_server_stats_t, p99_us);
    FIELD(cb_server_stats_t, arena_peak_bytes);
    FIELD(cb_server_stats_t, steps);
    SIZE(cb_tune_options_t);
    SIZE(cb_tune_candidate_t);
    FIELD(cb_tune_candidate_t, us);
    FIELD(cb_tune_candidate_t, row_reduce);
    SIZE(cb_tune_report_t);
    FIELD(cb_tune_report_t, cand);

    /* a 4 x 5 matrix, converted on the host and exported back */
    const int64_t rp[5] = {0, 2, 3, 3, 6};
    const int32_t ci[6] = {0, 4, 2, 1, 3, 4};
    const double va[6] = {1.5, -2.0, 3.25, 0.5, -1.0, 4.0};
    cb_options_t o;
    if (cb_options_default(&o) != CB_SUCCESS) return 2;
    cb_matrix_t A = NULL;
    if (cb_create_host(&A, 4, 5, 6, rp, ci, va, &o) != CB_SUCCESS) {
        printf("create failed: %s\n", cb_last_error());
        return 3;
    }
    cb_info_t info;
    info.struct_size = sizeof(info);
    if (cb_get_info(A, &info) != CB_SUCCESS) return 4;
    int64_t rp2[5];
    int32_t ci2[6];
    double va2[6];
    if (cb_export_csr(A, rp2, ci2, va2) != CB_SUCCESS) return 5;
    int same = 1;
    for (int i = 0; i < 5; ++i) same &= rp2[i] == rp[i];
    for (int i = 0; i < 6; ++i) same &= ci2[i] == ci[i] && va2[i] == va[i];
    printf("tiles %lld nnz %lld on_device %d roundtrip %s\n", (long long)info.ntiles, (long long)info.nnz,
           info.on_device, same ? "ok" : "MISMATCH");
    /* errors come back as statuses with a message */
    cb_matrix_t B = NULL;
    const int64_t bad[2] = {1, 0};
    const cb_status_t st = cb_create_host(&B, 1, 1, 0, bad, ci, va, NULL);
    printf("bad row_ptr status %d message %s\n", (int)st, cb_last_error()[0] ? "set" : "empty");
    cb_destroy(A);
    return same ? 0 : 1;
}
