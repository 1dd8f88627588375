"""MI355X-native block-space thread maps for discrete orthogonal m-simplex domains.

The work runs in hand-written HIP kernels (gfx950) behind the C ABI of
``include/simplexmap.h``; :mod:`paper_2208_11617_amd.binding` marshals
torch tensors and streams into it.  Import the binding explicitly:

    from paper_2208_11617_amd import binding as smap
    smap.map_launch(2, 1024, "accum", buf_in, buf_out)
"""
__all__ = ["binding", "build"]
