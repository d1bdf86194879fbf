"""Implicit surfaces and shape operations (Sec. III, "Implicit Surface
Representations" and "Calculus on Implicit Function Representations";
Listing 2).  TEST INFRASTRUCTURE ONLY: plain numpy definitions over the
oracle's grid, used by tests/ to check the library's device constructors.

Shapes, evaluated at every grid node x (coordinates from the oracle's grid):
  ball       sqrt(sum_{d in axes} (x_d - c_d)^2) - r: the signed distance to
             a sphere over every axis, or to a cylinder over a subset of them;
  ellipsoid  sum_{d in axes} w_d (x_d - c_d)^2 - r, Listing 2's form (a
             level-set function, not a distance).
Operations on two level-set functions (interiors where phi < 0):
  union min(a, b); intersection max(a, b); complement -a;
  subtraction (interior of a without that of b) max(a, -b).
"""
import numpy as np

from . import grid

SHAPES = {"ball": 0, "ellipsoid": 1}
OPS = {"union": 0, "intersection": 1, "complement": 2, "subtraction": 3}


def node_coords(P):
    """Coordinates of every node of problem P's grid, one array per axis."""
    axes = [grid(P, d)[1] for d in range(P.dim)]
    return np.meshgrid(*axes, indexing="ij")


def shape(P, kind, axes, center, radius, weights=None):
    X = node_coords(P)
    acc = np.zeros(X[0].shape)
    for d in axes:
        q = (X[d] - center[d]) ** 2
        acc = acc + (q if kind == "ball" else weights[d] * q)
    return (np.sqrt(acc) if kind == "ball" else acc) - radius


def op(name, a, b=None):
    if name == "union":
        return np.minimum(a, b)
    if name == "intersection":
        return np.maximum(a, b)
    if name == "complement":
        return -a
    if name == "subtraction":
        return np.maximum(a, -b)
    raise ValueError(name)
