// Device scratch for the entry point that allocates nothing (hc_join_count_noalloc).
//
// Each GPU the library runs on holds one file-scope array of kScratchBytes; its
// device address is looked up once per device (hipGetSymbolAddress, with that
// device current) when the first context on the device is created, and only that
// address is used afterwards.  A call carves its buffers out of the array with a
// first-fit arena kept on the host, so it makes no device allocation at all.
// Every call on a GPU shares that GPU's array: calls that overlap on one GPU race.
#include <mutex>

#include "hc_internal.h"

namespace hc {

constexpr size_t kScratchBytes = (size_t)256 << 20;   // 256 MiB per device
constexpr int kMaxDevices = 64;
constexpr size_t kScratchAlign = 256;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

void scratch_setup(int device) {
    HC_REQUIRE(device >= 0 && device < kMaxDevices, HC_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
        (void)hipGetLastError();
        fail(HC_ERR_DEVICE, std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(e));
    }
    g_scratch_ptr[device] = p;
}

void* scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

size_t scratch_bytes() { return kScratchBytes; }

// First-fit arena over [base, base + size): free ranges kept sorted by offset and
// coalesced on release.
ScratchArena::ScratchArena(void* base, size_t size) : base_((char*)base), size_(size) {
    free_.push_back({0, size});
}

void* ScratchArena::get(size_t bytes) {
    const size_t need = (bytes + kScratchAlign - 1) / kScratchAlign * kScratchAlign;
    for (size_t i = 0; i < free_.size(); ++i) {
        if (free_[i].len < need) continue;
        const size_t off = free_[i].off;
        free_[i].off += need;
        free_[i].len -= need;
        if (free_[i].len == 0) free_.erase(free_.begin() + (long)i);
        used_.push_back({off, need});
        if (off + need > high_) high_ = off + need;
        return base_ + off;
    }
    return nullptr;
}

void ScratchArena::put(void* p) {
    const size_t off = (size_t)((char*)p - base_);
    size_t len = 0;
    for (size_t i = 0; i < used_.size(); ++i)
        if (used_[i].off == off) {
            len = used_[i].len;
            used_.erase(used_.begin() + (long)i);
            break;
        }
    if (len == 0) return;
    size_t k = 0;
    while (k < free_.size() && free_[k].off < off) ++k;
    free_.insert(free_.begin() + (long)k, Range{off, len});
    if (k + 1 < free_.size() && free_[k].off + free_[k].len == free_[k + 1].off) {
        free_[k].len += free_[k + 1].len;
        free_.erase(free_.begin() + (long)k + 1);
    }
    if (k > 0 && free_[k - 1].off + free_[k - 1].len == free_[k].off) {
        free_[k - 1].len += free_[k].len;
        free_.erase(free_.begin() + (long)k);
    }
}

void* ScratchArena::alloc_cb(size_t bytes, void* user) { return static_cast<ScratchArena*>(user)->get(bytes); }
void ScratchArena::free_cb(void* p, void* user) { static_cast<ScratchArena*>(user)->put(p); }

}  // namespace hc
