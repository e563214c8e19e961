"""MI355X-native adaptive HEALPix ray-tracing radiative transfer (ARC, arXiv:1807.07094).

The compute path is the HIP library ``libarc.so`` behind the C ABI in ``include/arc.h``;
``paper_1807_07094_amd.arc`` is its thin ctypes binding. ``workload`` builds seeded
synthetic inputs. Importing the package does not load the GPU library.
"""
__version__ = "0.1.0"
