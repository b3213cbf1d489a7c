// Runtime services shared by the C ABI translation units (exs_api.cpp, exs_serve.cpp).
#pragma once

#include <stdint.h>

#include "exs.h"
#include "exs_internal.h"

namespace exs {
namespace rt {

int fail(int code, const char* fmt, ...);                 // sets the thread's last error
int current_device(int* dev);
int ensure_device(int dev);                               // once per device: tables, pool
int orientation_tables(int dev, int K, const float** r32, const double** r64);
int device_cus(int dev);

struct PocketInfo {
    int device = 0, channels = 0, storage = 0;
    GridDesc desc{};
};
bool pocket_info(int32_t id, PocketInfo* out);
void pocket_use(int32_t id, int delta);                   // pin / unpin against unload

// A validated persistent launch of an uploaded batch that allocates nothing: the launch
// arguments with the batch, pocket, search and order fields set (one work queue, the batch's
// upload-time order); the orientation table, outputs and every scratch pointer are left null.
struct NoAllocPlan {
    DockArgs args{};
    int device = 0, storage = 0, ppl = 1, threads = 64, resident = 1;
    size_t lds = 0;
    int64_t L = 0, A = 0, R = 0;
};
int noalloc_plan(int64_t batch, const exs_search_params* params, NoAllocPlan* out);

}  // namespace rt
}  // namespace exs
