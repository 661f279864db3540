"""Shared helpers of the GPU tests: move numpy interchange fields to the
device and back.  The library itself is reached only through its C ABI
(paper_0807_0264_amd.api)."""
import numpy as np
import torch

from paper_0807_0264_amd import api

F64, F32 = 0, 1


def links(U_np, prec):
    """numpy complex128 interchange field -> library Links of `prec`."""
    t = torch.from_numpy(np.ascontiguousarray(U_np)).cuda()
    return api.to_links(t, prec)


def gauge(G_np):
    return api.to_gauge(torch.from_numpy(np.ascontiguousarray(G_np)).cuda())


def host_links(W):
    """Library Links -> numpy complex128 interchange array (FP32 widened exactly)."""
    return api.from_links(W, torch.complex128).cpu().numpy()


def host_gauge(G):
    return api.from_gauge(G).cpu().numpy()


def rounded(U_np, prec):
    """The values a field of precision `prec` actually holds (what the oracle is fed)."""
    if prec == F64:
        return U_np
    return U_np.astype(np.complex64).astype(np.complex128)


def z_interchange(Z, L):
    """Library Z [4, V] (lexicographic) -> oracle layout [Lt, Lz, Ly, Lx, 4]."""
    z = Z.cpu().numpy().reshape(4, L[3], L[2], L[1], L[0])
    return np.ascontiguousarray(np.moveaxis(z, 0, -1))
