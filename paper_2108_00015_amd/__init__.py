"""MI355X-native ConKer hot path: mapping, shell convolution and n-point summation.

The compute runs in libconker.so (HIP, gfx950); this package only binds it to
PyTorch tensors.  See include/conker.h for the C ABI.
"""
from .api import (  # noqa: F401
    ConkerError,
    Context,
    Cosmology,
    Grid,
    Job,
    PRECISIONS,
    fused_supported,
    make_job,
    npcf_continuous,
    npcf_cross,
    npcf_diag,
    npcf_pair2,
    kspec_elems,
    npcf,
    num_tuples,
    shell_size,
)
