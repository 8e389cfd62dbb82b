"""MI355X-native RK4 interaction-picture step (Dennis, Hope & Johnsson, arXiv:1204.4255).

The compute path is the HIP library ``librk4ip.so`` built from ``csrc/``; ``rk4ip`` is
its ctypes binding. ``workloads`` builds the seeded synthetic inputs.
"""
