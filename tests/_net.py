"""Mapping between the oracle's network parameters and the library's padded
FP32 parameter vector (plumbing for the GPU network tests)."""
import numpy as np

from oracle import net as onet


def to_flat(params, layout, count):
    flat = np.zeros(count, dtype=np.float32)
    for (name, ci, co), L in zip(onet.LAYERS, layout):
        w = np.zeros((27, L["cout"], L["cin"]), dtype=np.float32)
        w[:, :co, :ci] = params[name + ".w"]
        flat[L["w_off"]:L["w_off"] + w.size] = w.ravel()
        bias = np.zeros(L["cout"], dtype=np.float32)
        bias[:co] = params[name + ".b"]
        flat[L["b_off"]:L["b_off"] + L["cout"]] = bias
    return flat


def from_flat(flat, layout):
    out = {}
    for (name, ci, co), L in zip(onet.LAYERS, layout):
        w = np.asarray(flat[L["w_off"]:L["w_off"] + 27 * L["cout"] * L["cin"]], dtype=np.float64)
        out[name + ".w"] = w.reshape(27, L["cout"], L["cin"])[:, :co, :ci].copy()
        out[name + ".b"] = np.asarray(flat[L["b_off"]:L["b_off"] + L["cout"]], dtype=np.float64)[:co].copy()
    return out


def padding_is_zero(flat, layout):
    ok = True
    for (name, ci, co), L in zip(onet.LAYERS, layout):
        w = np.asarray(flat[L["w_off"]:L["w_off"] + 27 * L["cout"] * L["cin"]]).reshape(27, L["cout"], L["cin"])
        ok &= not w[:, co:, :].any() and not w[:, :, ci:].any()
        ok &= not np.asarray(flat[L["b_off"] + co:L["b_off"] + L["cout"]]).any()
    return ok
