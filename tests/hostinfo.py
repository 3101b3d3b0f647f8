"""Host facts for the CPU-side legs (oracle timing and parity): how many threads the host
gives this process, and what the CPU is.  No part of the matrix-element arithmetic."""
import math
import os


def host_threads():
    """CPUs this process may use: the affinity mask, limited by a cgroup CPU quota if one is
    set (a container's share can be smaller than the mask)"""
    n = len(os.sched_getaffinity(0))
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            quota, period = f.read().split()[:2]
        if quota != "max":
            n = min(n, max(1, math.ceil(int(quota) / int(period))))
    except (OSError, ValueError):
        pass
    return n


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"
