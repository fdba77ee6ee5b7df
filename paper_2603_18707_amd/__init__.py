"""MI355X-native (gfx950) tile-based Gaussian splatting with the exponential or
ReLU-polynomial kernels of "From ex(p) to poly" and their tighter culling.

The compute path is libgs.so (HIP, built by ``python -m paper_2603_18707_amd.build``)
behind the C ABI in include/gs.h; ``_lib`` binds it with ctypes under the same
names, ``render`` drives the three forward stages, ``autograd`` wraps the
hand-written backward, ``scenes`` draws seeded synthetic inputs.
"""
__all__ = ["_lib", "render", "scenes"]
