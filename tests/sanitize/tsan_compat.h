// Force-included into the thread-sanitizer build of the server.  libstdc++
// implements std::condition_variable::wait_for / wait_until on the steady
// clock with pthread_cond_clockwait where glibc has it, and this gcc's thread
// sanitizer does not intercept that call: it then misses the mutex being
// released during the wait and reports double locks and races between threads
// that hold the mutex in turn.  Without the macro libstdc++ falls back to
// pthread_cond_timedwait, which the sanitizer understands.
#include <bits/c++config.h>
#undef _GLIBCXX_USE_PTHREAD_COND_CLOCKWAIT
