"""Device memory of the library from PyTorch's caching allocator (sbfem_set_allocator)."""

import torch

from . import binding


def use_torch_allocator():
    """Route the library's device allocations through torch.cuda's caching allocator."""
    def alloc(n):
        try:
            return torch.cuda.caching_allocator_alloc(n)
        except RuntimeError:  # out of memory: the library reports SBFEM_ENOMEM
            return 0

    binding.set_allocator(alloc, torch.cuda.caching_allocator_delete)


def use_hip_allocator():
    binding.set_allocator(None, None)
