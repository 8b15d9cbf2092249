"""Error measures of the parity tests.

Both relative measures of a result a against the reference b are taken, and a
test passes only when the larger of them is within the mode's tolerance:

* the 2-norm relative error      ||a - b||_2 / ||b||_2
* the element-wise bound         max_i |a_i - b_i| / ||b||_inf

The first alone lets a few badly wrong elements hide in a long vector; the
second catches them at the scale of the largest reference element.
"""
import numpy as np


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = a - b
    return max(float(np.linalg.norm(d) / np.linalg.norm(b)), float(np.abs(d).max() / np.abs(b).max()))


def rel_t(a, b):
    """The same for two torch tensors on one device, without copying them to the host."""
    import torch
    d = (a - b).double()
    bb = b.double()
    return max(float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(bb)),
               float(d.abs().max() / bb.abs().max()))
