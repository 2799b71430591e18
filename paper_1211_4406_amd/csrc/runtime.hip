// Runtime pieces of libsrf: error state, the device-memory cache, fill
// kernels and the device-wide exclusive scan.
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <map>
#include <mutex>
#include <vector>

#include "common.h"

namespace srf {

[[noreturn]] void fail(int status, const std::string& msg) { throw Error{status, msg}; }

void check_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return;
    if (e == hipErrorOutOfMemory) fail(SRF_ENOMEM, std::string(what) + ": out of device memory");
    fail(SRF_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ------------------------------------------------------------ memory cache
namespace {
struct Block {
    void* p;
    size_t bytes;
    hipStream_t stream;
};
struct Cache {
    std::mutex mu;
    std::multimap<std::pair<int, size_t>, Block> free_blocks;  // (device, bytes) -> block
    std::map<void*, std::pair<int, size_t>> live;              // ptr -> (device, bytes)
};
Cache& cache() {
    static Cache* c = new Cache();  // never destroyed: HIP may be gone at exit
    return *c;
}
size_t bucket(size_t bytes) {
    if (bytes <= 4096) {
        size_t b = 256;
        while (b < bytes) b <<= 1;
        return b;
    }
    if (bytes <= (size_t(1) << 22)) {  // <= 4 MiB: round up to 64 KiB
        return (bytes + 65535) & ~size_t(65535);
    }
    return (bytes + (size_t(2) << 20) - 1) & ~((size_t(2) << 20) - 1);  // 2 MiB granules
}
}  // namespace

void* dev_alloc(size_t bytes, hipStream_t stream) {
    int dev = 0;
    SRF_HIP(hipGetDevice(&dev));
    size_t b = bucket(bytes);
    Cache& c = cache();
    {
        std::lock_guard<std::mutex> lk(c.mu);
        auto it = c.free_blocks.lower_bound({dev, b});
        if (it != c.free_blocks.end() && it->first.first == dev && it->first.second <= b + b / 4) {
            Block blk = it->second;
            c.free_blocks.erase(it);
            c.live[blk.p] = {dev, blk.bytes};
            if (blk.stream != stream) {
                // last used on another stream: wait for that work to finish
                hipError_t e = hipStreamSynchronize(blk.stream);
                if (e != hipSuccess) {
                    c.live.erase(blk.p);
                    fail(SRF_EHIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
                }
            }
            return blk.p;
        }
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        dev_release_all();
        e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail(SRF_ENOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed");
        }
    }
    std::lock_guard<std::mutex> lk(c.mu);
    c.live[p] = {dev, b};
    return p;
}

void dev_free(void* p, hipStream_t stream) {
    if (!p) return;
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.live.find(p);
    if (it == c.live.end()) return;
    c.free_blocks.insert({it->second, Block{p, it->second.second, stream}});
    c.live.erase(it);
}

void dev_release_all() {
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    if (c.free_blocks.empty()) return;
    (void)hipDeviceSynchronize();
    for (auto& kv : c.free_blocks) (void)hipFree(kv.second.p);
    c.free_blocks.clear();
}

hipStream_t aux_stream() {
    static std::mutex mu;
    static std::map<int, hipStream_t>* streams = new std::map<int, hipStream_t>();   // never destroyed
    int dev = 0;
    SRF_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = streams->find(dev);
    if (it != streams->end()) return it->second;
    hipStream_t s = nullptr;
    SRF_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    (*streams)[dev] = s;
    return s;
}

void Tree::release_events() {
    for (hipEvent_t* e : {&gathered, &grouped})
        if (*e) (void)hipEventSynchronize(*e);
    for (hipEvent_t* e : {&sorted, &gathered, &sized, &grouped}) {
        if (*e) (void)hipEventDestroy(*e);
        *e = nullptr;
    }
}

// ------------------------------------------------------------------ fills
template <class T>
__global__ void k_fill(T* __restrict__ p, T v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, v, n);
    SRF_HIP(hipGetLastError());
}
void fill_f64(double* p, double v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, v, n);
    SRF_HIP(hipGetLastError());
}
void fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, v, n);
    SRF_HIP(hipGetLastError());
}

// ------------------------------------------------------------------- scan
// Blocks of 256 threads scan 2048 consecutive values (8 per thread); block
// totals are scanned recursively and added back.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

template <class T>
__device__ T wave_incl_scan(T v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// Exclusive scan of the thread-owned value across the block; returns the
// block total through `total`.
template <class T>
__device__ T block_excl_scan(T v, T* total) {
    __shared__ T wsum[kScanThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T incl = wave_incl_scan(v);
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) {
        T s = wsum[w];
        if (w < wid) off += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

// The tile goes through LDS: read and written by the block in coalesced
// rounds (value k * 256 + t by thread t), scanned as 8 consecutive values
// per thread.
template <class T>
__global__ __launch_bounds__(kScanThreads) void k_scan_local(T* __restrict__ data, int64_t n_read, int64_t n_write,
                                                             T* __restrict__ sums, const int32_t* __restrict__ nd) {
    __shared__ T buf[kScanTile];
    const int64_t b0 = (int64_t)blockIdx.x * kScanTile;
    if (nd) {   // a count on the device: scan its first *nd values, total at [*nd]
        n_read = *nd;
        n_write = n_read + 1;
        if (b0 >= n_write) {
            if (threadIdx.x == 0 && sums) sums[blockIdx.x] = T(0);
            return;
        }
    }
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = b0 + k * kScanThreads + threadIdx.x;
        buf[k * kScanThreads + threadIdx.x] = i < n_read ? data[i] : T(0);
    }
    __syncthreads();
    T v[kScanItems];
    T s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = buf[threadIdx.x * kScanItems + k];
        s += v[k];
    }
    T tot;
    T off = block_excl_scan(s, &tot);   // its barriers also order the reads above before the writes below
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        buf[threadIdx.x * kScanItems + k] = off;
        off += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = b0 + k * kScanThreads + threadIdx.x;
        if (i < n_write) data[i] = buf[k * kScanThreads + threadIdx.x];
    }
    if (threadIdx.x == 0 && sums) sums[blockIdx.x] = tot;
}

template <class T>
__global__ void k_scan_add(T* __restrict__ data, int64_t n, const T* __restrict__ sums,
                           const int32_t* __restrict__ nd) {
    if (nd) n = (int64_t)*nd + 1;
    const int64_t i = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
    const T add = sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t j = i + (int64_t)k * kScanThreads;
        if (j < n) data[j] += add;
    }
}

// With nd, n_write is the largest count + 1 the device may hold, and the
// top level scans the first *nd values (total at [*nd]).
template <class T>
static void scan_impl(T* data, int64_t n_read, int64_t n_write, hipStream_t s, const int32_t* nd = nullptr) {
    if (n_write <= 0) return;
    int64_t nb = (n_write + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_local<T>, dim3(1), dim3(kScanThreads), 0, s, data, n_read, n_write, (T*)nullptr,
                           nd);
        SRF_HIP(hipGetLastError());
        return;
    }
    DevBuf<T> sums(nb, s);
    hipLaunchKernelGGL(k_scan_local<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n_read, n_write,
                       sums.get(), nd);
    SRF_HIP(hipGetLastError());
    scan_impl<T>(sums.get(), nb, nb, s);
    hipLaunchKernelGGL(k_scan_add<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n_write,
                       (const T*)sums.get(), nd);
    SRF_HIP(hipGetLastError());
}

void exclusive_scan_i64(int64_t* data, int64_t n, bool write_total, hipStream_t s) {
    scan_impl<int64_t>(data, n, n + (write_total ? 1 : 0), s);
}
void exclusive_scan_i32_counted(int32_t* data, int64_t n_max, const int32_t* nd, hipStream_t s) {
    scan_impl<int32_t>(data, n_max, n_max + 1, s, nd);
}

}  // namespace srf
