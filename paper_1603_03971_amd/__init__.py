"""MI355X-native hot path of reverse time migration: radius-4 acoustic stencil time step with its
halo, pack and unpack phases, source injection, receiver recording and zero-lag imaging, in
hand-written HIP kernels behind the C ABI of ``librtm.so``."""
