// Storage of the emulated launch state and of the kernels' LDS arrays.
#include <hip/hip_runtime.h>
thread_local emu_idx blockIdx, threadIdx;
emu_idx blockDim, gridDim;
std::barrier<> *emu_bar = nullptr;
bool emu_capturing = false;
std::vector<std::function<void()>> emu_graph;
unsigned char emu_lds[1 << 18];
int emu_launches = 0;
bool emu_threaded = false;
namespace su3k { namespace p0 { alignas(16) unsigned char lds[1 << 18]; } namespace p1 { alignas(16) unsigned char lds[1 << 18]; } namespace p2 { alignas(16) unsigned char lds[1 << 18]; } namespace p3 { alignas(16) unsigned char lds[1 << 18]; } }
namespace su3k { char occupancy_reserve[1 << 16]; namespace p0 { char occupancy_reserve[1 << 16]; } namespace p1 { char occupancy_reserve[1 << 16]; } namespace p2 { char occupancy_reserve[1 << 16]; } namespace p3 { char occupancy_reserve[1 << 16]; } namespace dslash { alignas(16) char occupancy_reserve[160 << 10]; } namespace prog { char occupancy_reserve[1 << 16]; } }
