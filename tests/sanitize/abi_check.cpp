// abi_check.cpp -- drives the host side of the C ABI (include/pcgmi.h) for a
// host AddressSanitizer / UndefinedBehaviorSanitizer build of the library's
// host code (tests/test_sanitizers.py builds every source host-only and links
// this driver). It runs with no GPU and calls:
//   - every entry point with a null handle or null / out-of-range arguments,
//     which must return PCG_E_ARG with a message, before touching a device
//     (the destroy calls take NULL as a no-op);
//   - the creation calls, which must fail cleanly without a device (skipped
//     where a device is visible);
//   - pcg_sell_build, the host-only sliced-ELLPACK layout, on random
//     compressed-row matrices (empty rows, empty matrices, ragged last
//     chunks, several chunk and window sizes), checking the documented layout:
//     perm is a permutation, lengths decrease inside each sigma window (stable),
//     every stored entry appears once in its row's slots, padding is (-1, 0);
//     and on malformed inputs, which must be refused.
// Exit status 0 on success; the first failed check prints and exits 1.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "pcgmi.h"

#define CHECK(cond, ...)                                                 \
    do {                                                                 \
        if (!(cond)) {                                                   \
            std::fprintf(stderr, "abi_check: line %d: ", __LINE__);      \
            std::fprintf(stderr, __VA_ARGS__);                           \
            std::fputc('\n', stderr);                                    \
            std::exit(1);                                                \
        }                                                                \
    } while (0)

static void expect_arg(pcg_status st, const char* what) {
    CHECK(st == PCG_E_ARG, "%s: status %d, expected PCG_E_ARG", what, (int)st);
    const char* m = pcg_last_error();
    CHECK(m && std::strlen(m) > 0, "%s: no error message", what);
}

static uint64_t rng = 12345;
static uint32_t next_u32() {  // xorshift64* (Vigna 2016)
    rng ^= rng >> 12;
    rng ^= rng << 25;
    rng ^= rng >> 27;
    return (uint32_t)((rng * 0x2545F4914F6CDD1Dull) >> 32);
}

static void null_handles() {
    double d = 0;
    float f = 0;
    int i = 0;
    int64_t l = 0;
    pcg_info info;
    expect_arg(pcg_options_default(nullptr), "pcg_options_default");
    expect_arg(pcg_create(nullptr, 8, 8, 8, PCG_F32, nullptr, nullptr), "pcg_create(null out)");
    CHECK(pcg_destroy(nullptr) == PCG_OK, "pcg_destroy(NULL) is a no-op");
    expect_arg(stencil_apply(nullptr, &f, &f), "stencil_apply");
    expect_arg(axpy(nullptr, 1, 1.0, &f, &f, &f), "axpy");
    expect_arg(dot(nullptr, 1, &f, &f, &f), "dot");
    expect_arg(dot_f64(nullptr, 1, &f, &f, &d), "dot_f64");
    expect_arg(dot_noalloc(PCG_F32, -1, &f, &f, &f, nullptr, nullptr), "dot_noalloc(n < 0)");
    expect_arg(pcg_solve(nullptr, &f, &f, 1e-6, 10, &info), "pcg_solve");
    expect_arg(pcg_solve_refined(nullptr, &d, &d, 1e-6, 1e-2, 4, 10, &info), "pcg_solve_refined");
    expect_arg(pcg_refine_history(nullptr, &d, &i, 1, &i), "pcg_refine_history");
    expect_arg(pcg_set_coefficients(nullptr, &f), "pcg_set_coefficients");
    expect_arg(pcg_set_multigrid(nullptr, 1, 0.8, 8), "pcg_set_multigrid");
    expect_arg(pcg_mg_levels(nullptr, &i, &i), "pcg_mg_levels");
    expect_arg(pcg_mg_apply(nullptr, &f, &f), "pcg_mg_apply");
    expect_arg(pcg_solve_mg(nullptr, &f, &f, 1e-6, 10, &info), "pcg_solve_mg");
    expect_arg(pcg_get_history(nullptr, &d, 1, &i), "pcg_get_history");
    expect_arg(cnn_create(nullptr, nullptr), "cnn_create(null out)");
    CHECK(cnn_destroy(nullptr) == PCG_OK, "cnn_destroy(NULL) is a no-op");
    expect_arg(cnn_set_weights(nullptr, &f), "cnn_set_weights");
    expect_arg(cnn_get_weights(nullptr, &f), "cnn_get_weights");
    expect_arg(cnn_get_adam(nullptr, &f, &f, &l), "cnn_get_adam");
    expect_arg(cnn_set_adam(nullptr, &f, &f, 0), "cnn_set_adam");
    expect_arg(cnn_forward(nullptr, 8, 8, 8, PCG_F32, &f, &f, nullptr, &f), "cnn_forward");
    expect_arg(cnn_loss_grad(nullptr, 8, 8, 8, &f, &f, 1, &f, &d), "cnn_loss_grad");
    expect_arg(cnn_set_operator(nullptr, nullptr), "cnn_set_operator");
    expect_arg(cnn_set_loss_norm(nullptr, 0), "cnn_set_loss_norm");
    expect_arg(cnn_adam_step(nullptr, &f, 1e-3f), "cnn_adam_step");
    expect_arg(cnn_train_step(nullptr, 8, 8, 8, &f, &f, 1, 1e-3f, &d), "cnn_train_step");
    expect_arg(pcg_solve_flexible(nullptr, nullptr, &f, &f, &f, 1e-6, 10, &info), "pcg_solve_flexible");
    expect_arg(pcg_solve_snapshots(nullptr, &f, &f, 1e-6, 10, &i, 1, &f, &f, &info), "pcg_solve_snapshots");
    expect_arg(pcg_make_pairs(nullptr, 1, &d, &d, &d, &f), "pcg_make_pairs");
    expect_arg(pcg_batch_create(nullptr, 1, &i, nullptr, nullptr, 0, nullptr), "pcg_batch_create(null out)");
    CHECK(pcg_batch_destroy(nullptr) == PCG_OK, "pcg_batch_destroy(NULL) is a no-op");
    expect_arg(pcg_batch_layout(nullptr, &l, &l, &i, &i), "pcg_batch_layout");
    expect_arg(pcg_batch_set_barrier(nullptr, 0), "pcg_batch_set_barrier");
    expect_arg(pcg_batch_set_restarts(nullptr, 0), "pcg_batch_set_restarts");
    expect_arg(pcg_batch_solve(nullptr, &f, &d, 1e-6, 10, 0, &i, &d, &d, &i, &d), "pcg_batch_solve");
    expect_arg(pcg_sell_create(nullptr, 1, 1, &l, &i, &f, 1, nullptr), "pcg_sell_create(null out)");
    CHECK(pcg_sell_destroy(nullptr) == PCG_OK, "pcg_sell_destroy(NULL) is a no-op");
    expect_arg(pcg_sell_info(nullptr, &l, &l, &l), "pcg_sell_info");
    expect_arg(pcg_sell_spmv(nullptr, &f, &f), "pcg_sell_spmv");
    expect_arg(pcg_sell_solve(nullptr, &f, &d, 1e-6, 10, &info), "pcg_sell_solve");
    expect_arg(pcg_sell_set_graph(nullptr, 1), "pcg_sell_set_graph");
    expect_arg(pcg_sell_set_restarts(nullptr, 0), "pcg_sell_set_restarts");

    pcg_options o;
    CHECK(pcg_options_default(&o) == PCG_OK, "pcg_options_default");
}

// Without a device the creation calls fail and leave the out handle null.
static void no_device() {
    pcg_ctx c = reinterpret_cast<pcg_ctx>(1);
    pcg_status st = pcg_create(&c, 8, 8, 8, PCG_F32, nullptr, nullptr);
    CHECK(st != PCG_OK, "pcg_create without a device returned OK");
    CHECK(std::strlen(pcg_last_error()) > 0, "pcg_create: no message");
    expect_arg(pcg_create(&c, 0, 8, 8, PCG_F32, nullptr, nullptr), "pcg_create(nx = 0)");
    cnn_net n = nullptr;
    CHECK(cnn_create(&n, nullptr) != PCG_OK, "cnn_create without a device returned OK");
    int dims[3] = {8, 8, 8};
    pcg_batch b = nullptr;
    CHECK(pcg_batch_create(&b, 1, dims, nullptr, nullptr, 0, nullptr) != PCG_OK, "pcg_batch_create without a device");
    CHECK(cnn_num_weights() == 15120, "cnn_num_weights");
}

static void sell_case(int64_t nrows, int64_t ncols, int maxlen, int chunk, int sigma) {
    std::vector<int64_t> rowptr((size_t)nrows + 1, 0);
    for (int64_t r = 0; r < nrows; ++r) rowptr[r + 1] = rowptr[r] + (ncols > 0 ? next_u32() % (maxlen + 1) : 0);
    const int64_t nnz = rowptr[nrows];
    std::vector<int32_t> col((size_t)nnz);
    std::vector<float> val((size_t)nnz);
    for (int64_t k = 0; k < nnz; ++k) {
        col[k] = (int32_t)(next_u32() % ncols);
        val[k] = (float)(k + 1);  // unique: identifies the entry
    }
    int64_t nch = -1, nslots = -1;
    CHECK(pcg_sell_build(nrows, ncols, rowptr.data(), col.data(), val.data(), chunk, sigma, &nch, &nslots, nullptr,
                         nullptr, nullptr, nullptr) == PCG_OK, "sell sizes: %s", pcg_last_error());
    CHECK(nch == (nrows + chunk - 1) / chunk, "chunk count");
    // exact-size outputs, so that ASan sees any write past them
    std::vector<int64_t> cptr((size_t)nch + 1);
    int32_t* perm = (int32_t*)std::malloc(sizeof(int32_t) * (size_t)(nrows > 0 ? nrows : 1));
    int32_t* cout = (int32_t*)std::malloc(sizeof(int32_t) * (size_t)(nslots > 0 ? nslots : 1));
    float* vout = (float*)std::malloc(sizeof(float) * (size_t)(nslots > 0 ? nslots : 1));
    CHECK(pcg_sell_build(nrows, ncols, rowptr.data(), col.data(), val.data(), chunk, sigma, &nch, &nslots,
                         cptr.data(), perm, cout, vout) == PCG_OK, "sell layout: %s", pcg_last_error());
    CHECK(cptr[0] == 0 && cptr[nch] == nslots, "chunk pointers");
    std::vector<int> seen((size_t)nrows, 0);
    for (int64_t s = 0; s < nrows; ++s) {
        CHECK(perm[s] >= 0 && perm[s] < nrows && !seen[perm[s]], "perm is not a permutation");
        seen[perm[s]] = 1;
    }
    auto len = [&](int32_t r) { return rowptr[r + 1] - rowptr[r]; };
    for (int64_t s = 0; s + 1 < nrows; ++s) {
        const bool same_window = sigma > 1 && s / sigma == (s + 1) / sigma;
        if (same_window) {
            CHECK(len(perm[s]) >= len(perm[s + 1]), "lengths not decreasing in a window");
            if (len(perm[s]) == len(perm[s + 1])) CHECK(perm[s] < perm[s + 1], "sort not stable");
        } else if (sigma == 1) {
            CHECK(perm[s] == s, "sigma = 1 reorders rows");
        }
    }
    for (int64_t c = 0; c < nch; ++c) {
        const int64_t w = (cptr[c + 1] - cptr[c]) / chunk;
        CHECK((cptr[c + 1] - cptr[c]) % chunk == 0, "chunk width");
        for (int l = 0; l < chunk; ++l) {
            const int64_t s = c * chunk + l;
            const int64_t n = s < nrows ? len(perm[s]) : 0;
            for (int64_t j = 0; j < w; ++j) {
                const int64_t slot = cptr[c] + j * chunk + l;
                if (j < n) {
                    const int64_t k = rowptr[perm[s]] + j;
                    CHECK(cout[slot] == col[k] && vout[slot] == val[k], "entry %lld misplaced", (long long)k);
                } else {
                    CHECK(cout[slot] == -1 && vout[slot] == 0.0f, "padding slot");
                }
            }
        }
    }
    std::free(perm);
    std::free(cout);
    std::free(vout);
}

static void sell() {
    sell_case(0, 0, 0, 64, 1);
    sell_case(1, 1, 1, 64, 1);
    sell_case(63, 40, 5, 64, 1);
    sell_case(64, 64, 7, 64, 64);
    sell_case(65, 30, 9, 64, 128);
    sell_case(200, 200, 12, 4, 16);
    sell_case(257, 100, 3, 64, 256);
    sell_case(1000, 1000, 20, 8, 8);
    sell_case(37, 5, 0, 4, 4);  // no entries at all

    // malformed inputs
    int64_t nc, ns;
    const int64_t bad_ptr[3] = {0, 2, 1};
    const int32_t cols[2] = {0, 1};
    const float vals[2] = {1, 2};
    expect_arg(pcg_sell_build(2, 2, bad_ptr, cols, vals, 64, 1, &nc, &ns, nullptr, nullptr, nullptr, nullptr),
               "decreasing rowptr");
    const int64_t ptr1[3] = {1, 2, 2};
    expect_arg(pcg_sell_build(2, 2, ptr1, cols, vals, 64, 1, &nc, &ns, nullptr, nullptr, nullptr, nullptr),
               "rowptr[0] != 0");
    const int64_t ptr[3] = {0, 1, 2};
    const int32_t badcol[2] = {0, 2};
    expect_arg(pcg_sell_build(2, 2, ptr, badcol, vals, 64, 1, &nc, &ns, nullptr, nullptr, nullptr, nullptr),
               "column out of range");
    const int32_t negcol[2] = {-1, 0};
    expect_arg(pcg_sell_build(2, 2, ptr, negcol, vals, 64, 1, &nc, &ns, nullptr, nullptr, nullptr, nullptr),
               "negative column");
    expect_arg(pcg_sell_build(2, 2, ptr, cols, vals, 0, 1, &nc, &ns, nullptr, nullptr, nullptr, nullptr), "chunk 0");
    expect_arg(pcg_sell_build(2, 2, ptr, cols, vals, 64, 100, &nc, &ns, nullptr, nullptr, nullptr, nullptr),
               "sigma not a multiple of chunk");
    expect_arg(pcg_sell_build(-1, 2, ptr, cols, vals, 64, 1, &nc, &ns, nullptr, nullptr, nullptr, nullptr),
               "negative rows");
    expect_arg(pcg_sell_build((int64_t)1 << 31, 2, ptr, cols, vals, 64, 1, &nc, &ns, nullptr, nullptr, nullptr,
                              nullptr), "2^31 rows");
    expect_arg(pcg_sell_build(2, 2, nullptr, cols, vals, 64, 1, &nc, &ns, nullptr, nullptr, nullptr, nullptr),
               "null rowptr");
    expect_arg(pcg_sell_build(2, 2, ptr, nullptr, vals, 64, 1, &nc, &ns, nullptr, nullptr, nullptr, nullptr),
               "null columns");
    expect_arg(pcg_sell_build(2, 2, ptr, cols, vals, 64, 1, nullptr, &ns, nullptr, nullptr, nullptr, nullptr),
               "null count");
    int64_t cp[2];
    expect_arg(pcg_sell_build(2, 2, ptr, cols, vals, 64, 1, &nc, &ns, cp, nullptr, nullptr, nullptr),
               "partial outputs");
}

int main() {
    null_handles();
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) no_device();
    else std::puts("abi_check: a device is visible; the no-device checks are skipped");
    sell();
    std::puts("abi_check: ok");
    return 0;
}
