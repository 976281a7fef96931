// Enqueue a task on a stand-in stream (stub_runtime.cpp): tasks of one stream run in order
// on that stream's worker thread, after every task enqueued before them.
#pragma once
#include <functional>

#include <hip/hip_runtime.h>

void stub_enqueue(hipStream_t s, std::function<void()> task);
