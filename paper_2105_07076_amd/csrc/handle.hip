// handle.hip -- miid_create / miid_destroy, the per-device record and the
// tuning-table lookup.
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <set>
#include <utility>

#include "common.hpp"
#include "handle.hpp"

struct miid_handle_s {
    int device;  // -1: created without a visible device (workspace queries only)
    std::vector<miid::TuneRow> table;
};

namespace miid {

namespace {
constexpr int kMaxDevices = 64;

struct DevRecord {
    bool ready = false;
    int cus = 256;
};

std::mutex g_mu;
DevRecord g_dev[kMaxDevices];
std::set<std::pair<int, const void*>> g_lds_done;

int current_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();  // a host without a GPU: not an error of the call
        return -1;
    }
    return dev;
}

const char* kRoutineNames[] = {"id", "rid", "rid_sample", "two_sided", "cur", "batched"};

// One table row: "routine dtype m n k nb hints" (dtype f32 or f64; m, n, k
// of 0 match any value; hints decimal or 0x-hex).  Returns false on a
// malformed line.
bool parse_row(const char* line, TuneRow* r) {
    char name[32], dt[8];
    long long m, n, k, nb, hints;
    char tail[2];
    if (std::sscanf(line, "%31s %7s %lld %lld %lld %lld %lli %1s", name, dt, &m, &n, &k, &nb, &hints, tail) != 7)
        return false;
    int routine = -1;
    for (int i = 0; i < (int)(sizeof(kRoutineNames) / sizeof(kRoutineNames[0])); ++i)
        if (std::strcmp(name, kRoutineNames[i]) == 0) routine = i;
    if (routine < 0) return false;
    int dtype;
    if (std::strcmp(dt, "f32") == 0)
        dtype = MIID_F32;
    else if (std::strcmp(dt, "f64") == 0)
        dtype = MIID_F64;
    else
        return false;
    if (m < 0 || n < 0 || k < 0 || nb < 0 || nb > 64 || hints < 0 || (hints & ~(long long)kHintMask) != 0)
        return false;
    *r = TuneRow{routine, dtype, (int64_t)m, (int64_t)n, (int64_t)k, (int32_t)nb, (uint32_t)hints};
    return true;
}
}  // namespace

DevInfo dev_info() {
    const int dev = current_device();
    if (dev < 0) return DevInfo{-1, 256};
    std::lock_guard<std::mutex> lk(g_mu);
    DevRecord& r = g_dev[dev];
    if (!r.ready) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) r.cus = v;
        r.ready = true;
    }
    return DevInfo{dev, r.cus};
}

hipError_t lds_limit_once(const void* fn, int bytes) {
    const int dev = current_device();
    std::lock_guard<std::mutex> lk(g_mu);
    const auto key = std::make_pair(dev, fn);
    if (g_lds_done.count(key)) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess) g_lds_done.insert(key);
    return e;
}

int check_handle(miid_handle h) {
    if (!h || h->device < 0) return 0;
    const int dev = current_device();
    return (dev < 0 || dev == h->device) ? 0 : -1;
}

int resolve_opts(miid_handle h, int routine, miid_dtype dtype, int64_t m, int64_t n, int64_t k,
                 const miid_opts* in, miid_opts* out) {
    if (check_handle(h) != 0) return -1;
    if (!in) return 0;  // the body reports the missing options
    *out = *in;
    if (!h || in->nb != 0 || (in->flags & kHintMask) != 0) return 0;
    const TuneRow* best = nullptr;
    int best_spec = -1;
    for (const TuneRow& r : h->table) {
        if (r.routine != routine || r.dtype != (int)dtype) continue;
        if ((r.m && r.m != m) || (r.n && r.n != n) || (r.k && r.k != k)) continue;
        const int spec = (r.m != 0) + (r.n != 0) + (r.k != 0);
        if (spec > best_spec) {
            best = &r;
            best_spec = spec;
        }
    }
    if (best) {
        out->nb = best->nb;
        out->flags |= best->hints;
    }
    return 0;
}

}  // namespace miid

using namespace miid;

extern "C" {

int miid_create(miid_handle* out, const char* autotune_path) {
    if (!out) return -1;
    *out = nullptr;
    std::vector<TuneRow> table;
    if (autotune_path) {
        FILE* f = std::fopen(autotune_path, "r");
        if (!f) return -2;
        char line[512];
        bool ok = true;
        while (std::fgets(line, sizeof line, f)) {
            const char* s = line;
            while (*s == ' ' || *s == '\t') ++s;
            if (*s == '#' || *s == '\n' || *s == '\r' || *s == '\0') continue;
            TuneRow r;
            if (!parse_row(s, &r)) {
                ok = false;
                break;
            }
            table.push_back(r);
        }
        std::fclose(f);
        if (!ok) return -2;
    }
    const DevInfo d = dev_info();  // fills the device record once
    // the set-up of this device's allocation-free scratch (its address)
    if (d.device >= 0) {
        const int rc = batched_noalloc_setup();
        if (rc != 0) return rc;
    }
    miid_handle h = new (std::nothrow) miid_handle_s;
    if (!h) return MIID_E_UNSUPPORTED;
    h->device = d.device;
    h->table = std::move(table);
    *out = h;
    return 0;
}

void miid_destroy(miid_handle h) { delete h; }

int miid_handle_device(miid_handle h) { return h ? h->device : -1; }

int miid_handle_rows(miid_handle h) { return h ? (int)h->table.size() : 0; }

}  // extern "C"
